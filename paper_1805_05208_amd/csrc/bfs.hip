// Single-source BFS: frontier rounds of edgeMap with a sparse (push) / dense
// (pull) switch decided on the device every round.
//
// Method (paper: BFS algorithm box; edgeMap in Preliminaries, "Ligra, Ligra+,
// and Julienne"; blocked sparse traversal in the "edgeMapBlocked" section):
//   round r processes the frontier U_r (vertices at distance r) and produces
//   U_{r+1}.  Sparse rounds walk the frontier's edges in edge-balanced blocks;
//   dense rounds let every unvisited vertex scan its own (in-)edges in order
//   and stop at the first frontier neighbour.  The switch goes dense when
//   |U| + sum deg(U) exceeds m / tau.
// Determinism: the paper's test-and-set leaves the parent to a race; here
//   push rounds take atomicMin over frontier neighbours and dense rounds scan
//   ascending lists and stop at the first hit, so both give
//   parent[v] = min{u in N(v) : D[u] = D[v] - 1} and the direction schedule
//   never changes the result.
//
// Device state (all words are uint32):
//   V        visited bitmap (vertices of distance < r, plus degree-0 vertices)
//   F[3]     frontier bitmaps; F[r%3] = U_r, F[(r+1)%3] receives U_{r+1},
//            F[(r+2)%3] is cleared during round r for round r+1
//   Q[2],P[2] sparse frontier: vertex ids and exclusive degree prefix sums
//   cnt[4]   per-round totals, (|U_r| << 32) | sum deg(U_r)
//   qcnt[4]  per-round queue reservations, same packing
//   qover[4] 1 when round r's queue was abandoned (too large to be useful)
// A vertex is "visited for round r" when V | F[r%3] has its bit; V is folded
// with U_r during round r without changing that union.

#include "common.h"
#include "emit.h"
#include "gridbar.h"

namespace gb {

static size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

// The control block: 64 words of counters, the round totals (4 slots of
// kSpread spread counters), then the grid-barrier area of the single-launch
// form (kBarWords 32-bit words).
constexpr int kCtlWords = 64 + 4 * kSpread * kSpreadStride;

size_t bfs_ws_bytes(int64_t n, int64_t nwords) {
    return al256((size_t)nwords * 4) * 4 + al256((size_t)(n + 64) * 4) * 4 +
           al256((size_t)kCtlWords * 8 + (size_t)kBarWords * 4);
}

// Points the workspace at `mem` (bfs_ws_bytes(n, nwords) bytes of device
// memory).  The memory stays owned by the caller.
void bfs_ws_attach(BfsWs* w, void* mem, int64_t n, int64_t nwords) {
    w->n = n;
    w->nwords = nwords;
    char* p = (char*)mem;
    w->V = (uint32_t*)p; p += al256((size_t)nwords * 4);
    for (int i = 0; i < 3; ++i) { w->F[i] = (uint32_t*)p; p += al256((size_t)nwords * 4); }
    for (int i = 0; i < 2; ++i) { w->Q[i] = (uint32_t*)p; p += al256((size_t)(n + 64) * 4); }
    for (int i = 0; i < 2; ++i) { w->P[i] = (uint32_t*)p; p += al256((size_t)(n + 64) * 4); }
    w->ctl = (unsigned long long*)p;
}

// Host-side parts: pinned progress / log words and timing events.
int bfs_ws_host_init(BfsWs* w) {
    GB_TRY(host_log_alloc(&w->hl, kLogCap));
    if (hipEventCreate(&w->ev0) != hipSuccess || hipEventCreate(&w->ev1) != hipSuccess ||
        hipEventCreateWithFlags(&w->done, hipEventDisableTiming) != hipSuccess)
        return set_error(GBGPU_E_HIP, "BFS workspace: event creation failed");
    return GBGPU_OK;
}

BfsWs* bfs_ws_new() { return new BfsWs(); }

void free_bfs_ws(BfsWs* w) {
    if (!w) return;
    if (w->block) (void)hipFree(w->block);
    if (w->done) {
        (void)hipEventSynchronize(w->done);  // launches of the last run may still be queued
        (void)hipEventDestroy(w->done);
    }
    host_log_free(&w->hl);
    if (w->ev0) (void)hipEventDestroy(w->ev0);
    if (w->ev1) (void)hipEventDestroy(w->ev1);
    delete w;
}

static int ensure_bfs_ws(gbgpu_graph g) {
    if (g->bfs) return GBGPU_OK;
    BfsWs* w = new BfsWs();
    const size_t total = bfs_ws_bytes(g->n, g->nwords);
    hipError_t e = hipMalloc(&w->block, total);
    if (e != hipSuccess) {
        delete w;
        return set_error(GBGPU_E_NOMEM, "BFS workspace of %zu bytes: %s", total,
                         hipGetErrorString(e));
    }
    bfs_ws_attach(w, w->block, g->n, g->nwords);
    int s = bfs_ws_host_init(w);
    if (s != GBGPU_OK) {
        free_bfs_ws(w);
        return s;
    }
    g->bfs = w;
    return GBGPU_OK;
}

__device__ __forceinline__ uint32_t* bfs_bar(unsigned long long* ctl) {
    return reinterpret_cast<uint32_t*>(ctl + kCtlWords);
}

struct BfsArgs {
    const int64_t* off;
    const int32_t* nbr;
    const uint32_t* deg;
    uint32_t* V;
    uint32_t* F0;
    uint32_t* F1;
    uint32_t* F2;
    uint32_t* Q0;
    uint32_t* Q1;
    uint32_t* P0;
    uint32_t* P1;
    int32_t* dist;
    uint32_t* parent;
    unsigned long long* ctl;
    uint32_t* prog;         // host progress words (device address)
    uint32_t* log;          // host round log (device address)
    const uint4* head;      // first four neighbours of each vertex
    const uint32_t* nz;     // vertices of degree >= 2 (the ones dense rounds scan)
    const uint4* nz_head;   // their head records, in the same order
    uint32_t nnz;
    const uint2* leaf;      // (vertex of degree 1, its one neighbour)
    uint32_t nleaf;
    uint32_t src;
    uint32_t m32;           // number of stored edges
    int64_t n;
    int64_t nwords;
    uint64_t dense_thresh;  // go dense when |U| + sum deg(U) > dense_thresh
    uint32_t stay_dense;    // after a dense round, stay dense while |U| > stay_dense
    int32_t force_dir;
    int32_t light;
    uint32_t chunk_cap;
};

// ---------------------------------------------------------------------------
// init: dist = INF, parent = -1, V = zero-degree mask, F = {src}, Q = [src]
// ---------------------------------------------------------------------------
// x[0, n) = val except x[sp] = spval, in 16-byte stores from the first
// 16-byte boundary on (the caller's arrays are only 4-byte aligned).
__device__ __forceinline__ void fill_u32(uint32_t* x, int64_t n, uint32_t val, int64_t sp,
                                         uint32_t spval, int64_t tid, int64_t stride) {
    const int64_t head = min<int64_t>(n, (int64_t)(((16u - ((uintptr_t)x & 15u)) & 15u) >> 2));
    if (tid < head) x[tid] = tid == sp ? spval : val;
    const int64_t nv = (n - head) >> 2;
    uint4* xv = reinterpret_cast<uint4*>(x + head);
    for (int64_t i = tid; i < nv; i += stride) {
        const int64_t b = head + 4 * i;
        uint4 q;
        q.x = sp == b ? spval : val;
        q.y = sp == b + 1 ? spval : val;
        q.z = sp == b + 2 ? spval : val;
        q.w = sp == b + 3 ? spval : val;
        xv[i] = q;
    }
    const int64_t t0 = head + 4 * nv;
    if (tid < n - t0) x[t0 + tid] = t0 + tid == sp ? spval : val;
}

__global__ __launch_bounds__(kBlock) void bfs_init_kernel(BfsArgs a, const uint32_t* pruned,
                                                          uint32_t src) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    fill_u32(reinterpret_cast<uint32_t*>(a.dist), a.n, (uint32_t)INT32_MAX, src, 0u, tid, stride);
    fill_u32(a.parent, a.n, kNone, src, src, tid, stride);
    for (int64_t w = tid; w < a.nwords; w += stride) {
        a.V[w] = pruned[w];
        a.F0[w] = (w == (int64_t)(src >> 5)) ? (1u << (src & 31)) : 0u;
        a.F1[w] = 0u;
        a.F2[w] = 0u;
    }
    if (tid == 0) {
        a.Q0[0] = src;
        a.P0[0] = 0;
        unsigned long long* qcnt = a.ctl + 4;
        unsigned long long* qover = a.ctl + 8;
        const uint32_t src_deg = a.deg[src];
        qcnt[0] = (1ull << 32) | src_deg;
        for (int i = 1; i < 4; ++i) qcnt[i] = 0;
        for (int i = 0; i < 4; ++i) qover[i] = 0;
        a.ctl[13] = 0;  // workgroups done with the leaf pass
        a.ctl[16] = 0;  // leaves reached
        a.ctl[17] = 0;  // largest leaf distance
        a.ctl[14] = 0;  // vertices reached through round r - 1, by parity of r
        a.ctl[15] = 0;
    }
    // grid barrier of the single-launch form: every count, flag and the
    // abort word start at zero
    uint32_t* bar = bfs_bar(a.ctl);
    for (int64_t i = tid; i < kBarWords; i += stride) bar[i] = 0u;
    // round totals: 4 slots of kSpread counters; slot 0 holds U_0 = {src}
    unsigned long long* tot = a.ctl + 64;
    for (int64_t i = tid; i < 4 * kSpread; i += stride)
        tot[i * kSpreadStride] = i == 0 ? ((1ull << 32) | a.deg[src]) : 0ull;
}

// Sparse-round edge operation: claim v for round r+1 with the smallest
// frontier neighbour as parent (check-before-atomic, then atomicMin).
struct PushPolicy {
    const BfsArgs* a;
    const uint32_t* Fc;
    uint32_t* Fn;
    WgQueue* q;
    const QueueOut* out;
    uint32_t r;
    static constexpr bool kSkipDead = false;

    __device__ __forceinline__ uint32_t aux(uint32_t) const { return 1u; }

    __device__ __forceinline__ void edge(bool act, uint32_t u, uint32_t, int64_t e, bool) {
        bool claim = false;
        uint32_t v = 0, dv = 0;
        if (act) {
            v = (uint32_t)a->nbr[e];
            const uint32_t w = v >> 5, bit = 1u << (v & 31);
            if (!((a->V[w] | Fc[w]) & bit)) {
                uint32_t pv = a->parent[v];
                if (u < pv) {
                    uint32_t old = atomicMin(&a->parent[v], u);
                    if (old == kNone) {
                        claim = true;
                        a->dist[v] = (int32_t)(r + 1);
                        atomicOr(&Fn[w], bit);
                        dv = a->deg[v];
                    }
                }
            }
        }
        wgq_push(*q, claim, v, dv, *out);
    }

    __device__ __forceinline__ void window_done() {}
};

// Direction of round r.  A frontier without a queue (it came out of a dense
// round) stays dense while it holds more than stay_dense vertices, even when
// its edges are few: the push would touch one list per frontier vertex,
// while the pull only revisits the still unvisited vertices.
__device__ __forceinline__ bool choose_push(const BfsArgs& a, uint32_t r, uint32_t count,
                                            uint32_t edges, bool qvalid) {
    if (a.force_dir == 1) return true;
    if (a.force_dir == 2) return false;
    if (a.force_dir == 3) return (r & 1u) == 0u;
    if (!qvalid && count > a.stay_dense) return false;
    return (uint64_t)count + edges <= a.dense_thresh;
}

// Dense (pull) processing: each unvisited vertex scans its list in ascending
// order and stops at the first member of the frontier, which is its parent.
// A wavefront holds kPullG x 64 candidates at a time (lane l owns candidates
// l + 64 j).  The rounds are bound by scattered requests in flight per CU,
// not by registers, so one candidate per lane is the fastest setting (more
// per lane lengthens every wavefront's slowest chain).
constexpr int kPullG = 1;
// four neighbours in one load; list starts are only 4-byte aligned
typedef uint32_t u32x4_a4 __attribute__((ext_vector_type(4), aligned(4)));

// Scans kPullG x 64 candidate vertices held by the lanes (v[j] ascending
// with the lane index for each j; in[j] false for empty slots).  With kCheck
// the candidates are first tested against V | F_r; without it they are known
// to be unvisited.
template <bool kCheck>
__device__ __forceinline__ void pull_vertices(const BfsArgs& a, uint32_t r,
                                              const uint32_t (&v)[kPullG], const uint32_t (&hi)[kPullG],
                                              const bool (&in)[kPullG],
                                              const uint32_t* __restrict__ Fc, uint32_t* Fn,
                                              uint32_t& found, uint32_t& dsum) {
    const int l = lane_id();
    // 1. the first four neighbours come from the list-head records (one
    //    coalesced 16-byte load per vertex); the first alone decides most
    //    vertices
    uint4 h4[kPullG];
    uint32_t hit[kPullG];
    bool unvis[kPullG];
    bool any_unvis = false;
#pragma unroll
    for (int j = 0; j < kPullG; ++j) {
        // list candidates read their head record by list position, so the
        // load needs neither the vertex id nor the visited test first
        uint32_t vw = 0u;
        uint4 hh = make_uint4(kNone, kNone, kNone, kNone);
        if (in[j]) hh = kCheck ? a.nz_head[hi[j]] : a.head[hi[j]];
        if constexpr (kCheck) {
            if (in[j]) vw = a.V[v[j] >> 5] | Fc[v[j] >> 5];
        }
        unvis[j] = in[j] && !((vw >> (v[j] & 31)) & 1u);
        h4[j] = unvis[j] ? hh : make_uint4(kNone, kNone, kNone, kNone);
        hit[j] = kNone;
        any_unvis |= unvis[j];
    }
    if (ballot(any_unvis) == 0) return;
#pragma unroll
    for (int j = 0; j < kPullG; ++j)
        if (h4[j].x != kNone && test_bit(Fc, h4[j].x)) hit[j] = h4[j].x;
#pragma unroll
    for (int j = 0; j < kPullG; ++j) {
        if (hit[j] == kNone && h4[j].y != kNone) {
            // one bit test at a time: fewer scattered requests, and most of
            // these vertices stop at the second neighbour
            if (test_bit(Fc, h4[j].y)) hit[j] = h4[j].y;
            else if (h4[j].z != kNone && test_bit(Fc, h4[j].z)) hit[j] = h4[j].z;
            else if (h4[j].w != kNone && test_bit(Fc, h4[j].w)) hit[j] = h4[j].w;
        }
    }
    // 2. vertices with more than four neighbours and no hit yet continue in
    //    the list itself.  Edge indices fit in 32 bits (m < 2^31); a
    //    vertex that does not continue gets k = lim = e.
    uint32_t e[kPullG], k[kPullG], lim[kPullG];
#pragma unroll
    for (int j = 0; j < kPullG; ++j) {
        const bool more = unvis[j] && hit[j] == kNone && h4[j].w != kNone;
        uint32_t s0 = 0, e0 = 0;
        if (more) {
            s0 = (uint32_t)a.off[v[j]] + 4u;
            e0 = (uint32_t)a.off[v[j] + 1];
        }
        e[j] = more ? e0 : 0u;
        k[j] = more ? s0 : 0u;
        lim[j] = more ? min(e0, s0 + a.light) : 0u;
    }
    // light phase: lanes scan up to `light` neighbours of each of their
    // vertices, four at a time (one 16-byte load), in ascending order
    for (;;) {
        bool act[kPullG];
        bool any_act = false;
#pragma unroll
        for (int j = 0; j < kPullG; ++j) {
            act[j] = k[j] < lim[j] && hit[j] == kNone;
            any_act |= act[j];
        }
        if (!any_act) break;
        uint32_t u[kPullG][4];
#pragma unroll
        for (int j = 0; j < kPullG; ++j) {
            if (act[j] && k[j] + 4u <= a.m32) {
                const u32x4_a4 q4 = *(const u32x4_a4*)(a.nbr + k[j]);
                u[j][0] = q4.x;
                u[j][1] = q4.y;
                u[j][2] = q4.z;
                u[j][3] = q4.w;
            } else {
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    u[j][i] = (act[j] && k[j] + i < a.m32) ? (uint32_t)a.nbr[k[j] + i] : kNone;
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (!act[j] || k[j] + i >= lim[j]) u[j][i] = kNone;
        }
#pragma unroll
        for (int j = 0; j < kPullG; ++j) {
            if (act[j]) {
                uint32_t hj = kNone;
#pragma unroll
                for (int i = 3; i >= 0; --i)
                    if (u[j][i] != kNone && test_bit(Fc, u[j][i])) hj = u[j][i];
                hit[j] = hj;
                k[j] += 4;
            }
        }
    }
    // heavy phase: vertices with neighbours left are scanned by the whole
    // wavefront, 128 neighbours per step, first hit wins
#pragma unroll
    for (int j = 0; j < kPullG; ++j) {
        uint64_t hm = ballot(hit[j] == kNone && lim[j] < e[j]);
        while (hm) {
            const int hl = first_lane(hm);
            hm &= hm - 1;
            const int64_t hs = (int64_t)__shfl(lim[j], hl, 64);
            const int64_t he = (int64_t)__shfl(e[j], hl, 64);
            uint32_t fu = kNone;
            for (int64_t b = hs; b < he; b += 128) {
                const int64_t i0 = b + l, i1 = b + 64 + l;
                const uint32_t u0 = i0 < he ? (uint32_t)a.nbr[i0] : 0u;
                const uint32_t u1 = i1 < he ? (uint32_t)a.nbr[i1] : 0u;
                const bool h0 = i0 < he && test_bit(Fc, u0);
                const bool h1 = i1 < he && test_bit(Fc, u1);
                const uint64_t b0 = ballot(h0);
                if (b0) {
                    fu = __shfl(u0, first_lane(b0), 64);
                    break;
                }
                const uint64_t b1 = ballot(h1);
                if (b1) {
                    fu = __shfl(u1, first_lane(b1), 64);
                    break;
                }
            }
            if (l == hl) hit[j] = fu;
        }
    }
#pragma unroll
    for (int j = 0; j < kPullG; ++j) {
        const bool f = hit[j] != kNone;
        if (f) {
            a.dist[v[j]] = (int32_t)(r + 1);
            a.parent[v[j]] = hit[j];
            found += 1;
            dsum += a.deg[v[j]];
        }
        // the lanes' vertices ascend with the lane index, so lanes sharing a
        // bitmap word are adjacent: OR their bits towards the first lane of
        // each run and let that lane alone write the word
        const uint32_t wd = in[j] ? v[j] >> 5 : 0xFFFFFFFFu;
        uint32_t bits = f ? 1u << (v[j] & 31) : 0u;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t ob = __shfl_down(bits, d, 64);
            const uint32_t ow = __shfl_down(wd, d, 64);
            if (l + d < 64 && ow == wd) bits |= ob;
        }
        const uint32_t pw = __shfl_up(wd, 1, 64);
        if (bits && (l == 0 || pw != wd)) atomicOr(&Fn[wd], bits);
    }
}

// Dense pass over the list of vertices of nonzero degree: every wavefront
// takes kPullG x 64 consecutive entries at a time (balanced when most of them
// are still unvisited).
__device__ __forceinline__ void pull_list(const BfsArgs& a, uint32_t r, uint32_t gwave,
                                          uint32_t nwaves, const uint32_t* __restrict__ Fc,
                                          uint32_t* Fn, uint32_t* Fclr, uint32_t& found,
                                          uint32_t& dsum) {
    // fold U_r into V (leaves V | F_r unchanged) and clear the bitmap that
    // round r+1 writes
    for (int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w < a.nwords;
         w += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t fw = Fc[w];
        if (fw) a.V[w] |= fw;
        Fclr[w] = 0u;
    }
    const int l = lane_id();
    const uint32_t per = 64u * kPullG;
    for (uint32_t base = gwave * per; base < a.nnz; base += nwaves * per) {
        uint32_t v[kPullG], hi[kPullG];
        bool in[kPullG];
#pragma unroll
        for (int j = 0; j < kPullG; ++j) {
            const uint32_t i = base + (uint32_t)l + 64u * j;
            in[j] = i < a.nnz;
            v[j] = in[j] ? a.nz[i] : 0u;
            hi[j] = i;
        }
        pull_vertices<true>(a, r, v, hi, in, Fc, Fn, found, dsum);
    }
}

// Dense pass over the unvisited bitmap ~(V | F_r) (degree-0 vertices are
// in V from the start): every wavefront takes 64 words (2048 vertex ids) at
// a time, folds U_r into V and clears round r+1's bitmap for them, and
// scans the unvisited ids it finds, kPullG x 64 at a time in ascending
// order.  Cheaper than the list once few vertices remain unvisited.
__device__ __forceinline__ void pull_bitmap(const BfsArgs& a, uint32_t r, uint32_t gwave,
                                            uint32_t nwaves, const uint32_t* __restrict__ Fc,
                                            uint32_t* Fn, uint32_t* Fclr, uint32_t& found,
                                            uint32_t& dsum) {
    const int l = lane_id();
    const int64_t nblk = (a.nwords + 63) / 64;
    for (int64_t blk = gwave; blk < nblk; blk += nwaves) {
        const int64_t w = blk * 64 + l;
        uint32_t x = 0u;
        if (w < a.nwords) {
            const uint32_t fw = Fc[w];
            const uint32_t vw = a.V[w];
            if (fw) a.V[w] = vw | fw;
            Fclr[w] = 0u;
            const int64_t v0 = w * 32;
            x = ~(vw | fw);
            if (v0 >= a.n) x = 0u;
            else if (v0 + 32 > a.n) x &= (1u << (uint32_t)(a.n - v0)) - 1u;
        }
        const uint32_t c = (uint32_t)__popc(x);
        const uint32_t inc = wave_incl_sum(c);
        const uint32_t total = __shfl(inc, 63, 64);
        const uint32_t excl = inc - c;
        for (uint32_t B = 0; B < total; B += 64u * kPullG) {
            uint32_t v[kPullG];
            bool in[kPullG];
#pragma unroll
            for (int j = 0; j < kPullG; ++j) {
                const uint32_t idx = B + (uint32_t)l + 64u * j;
                in[j] = idx < total;
                int o = 0;
#pragma unroll
                for (int s = 32; s >= 1; s >>= 1) {
                    const uint32_t pv = __shfl(excl, o + s, 64);
                    if (pv <= idx) o += s;
                }
                const uint32_t xo = __shfl(x, o, 64);
                const uint32_t k = idx - __shfl(excl, o, 64);
                v[j] = in[j] ? (uint32_t)((blk * 64 + o) * 32) + select_bit(xo, k) : 0u;
            }
            pull_vertices<false>(a, r, v, v, in, Fc, Fn, found, dsum);
        }
    }
}

// Degree-1 vertices take no part in the rounds (they start in V): such a
// vertex can only be reached through its one neighbour u and is never the
// parent of anyone else, so after the last round D[v] = D[u] + 1 and
// parent[v] = u whenever u was reached.  The last workgroup to finish this
// pass reports the end of the BFS to the host.
constexpr int kLeafBatch = 8;

__device__ __forceinline__ void attach_leaves(const BfsArgs& a, uint32_t r, WgQueue& q) {
    // kLeafBatch records per thread and pass, every load of a pass issued
    // before its first store: one round trip for the records and one for
    // the neighbours' distances per pass, instead of two per leaf.  A leaf's
    // neighbour is never a leaf that this pass writes (it is either of
    // degree >= 2, finished by the rounds, or a degree-1 source, skipped
    // here), so reading dist ahead of the stores is safe.
    uint32_t reached = 0, deepest = 0;
    const uint32_t nthreads = gridDim.x * blockDim.x;
    for (uint32_t base = blockIdx.x * blockDim.x + threadIdx.x; base < a.nleaf;
         base += kLeafBatch * nthreads) {
        uint2 rec[kLeafBatch];
        int32_t du[kLeafBatch];
#pragma unroll
        for (int j = 0; j < kLeafBatch; ++j) {
            const uint32_t i = base + (uint32_t)j * nthreads;
            rec[j] = i < a.nleaf ? a.leaf[i] : make_uint2(a.src, a.src);
        }
#pragma unroll
        for (int j = 0; j < kLeafBatch; ++j)
            du[j] = rec[j].x == a.src ? INT32_MAX : a.dist[rec[j].y];
#pragma unroll
        for (int j = 0; j < kLeafBatch; ++j) {
            if (du[j] != INT32_MAX) {
                a.dist[rec[j].x] = du[j] + 1;
                a.parent[rec[j].x] = rec[j].y;
                ++reached;
                deepest = max(deepest, (uint32_t)du[j] + 1u);
            }
        }
    }
    reached = wave_sum(reached);
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) deepest = max(deepest, (uint32_t)__shfl_xor(deepest, d, 64));
    if (lane_id() == 0 && reached) {
        atomicAdd(&q.found, reached);
        atomicMax(&q.fdsum, deepest);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (q.found) {
            atomicAdd(&a.ctl[16], (unsigned long long)q.found);
            atomicMax(&a.ctl[17], (unsigned long long)q.fdsum);
        }
        __threadfence();
        const unsigned long long done = atomicAdd(&a.ctl[13], 1ull);
        if (done == gridDim.x - 1) {
            __threadfence();
            host_store(&a.prog[2], (uint32_t)atomicAdd(&a.ctl[16], 0ull));
            host_store(&a.prog[3], (uint32_t)atomicMax(&a.ctl[17], 0ull));
            __threadfence_system();
            host_store(&a.prog[1], r + 1);
        }
    }
}

// One BFS round (workgroup-uniform); returns true when round r found the
// frontier empty (the search is over: the first such round attached the
// degree-1 vertices and told the host).
__device__ __forceinline__ bool bfs_round(const BfsArgs& a, uint32_t r, WgQueue& q,
                                          unsigned long long& s_tot, unsigned long long& s_prev) {
    unsigned long long* qcnt = a.ctl + 4;
    unsigned long long* qover = a.ctl + 8;
    unsigned long long* tot = a.ctl + 64;  // 4 slots x kSpread x kSpreadStride
    const uint32_t rs = r & 3u;
    // written by earlier rounds and independent of the totals: loaded with
    // them, one trip before the workgroup barrier instead of one after it
    const unsigned long long reached_before = a.ctl[14 + ((r + 1) & 1u)];
    const unsigned long long qover_r = qover[rs];
    if (threadIdx.x < kWave) {
        const unsigned long long t = spread_sum(tot + (size_t)rs * kSpread * kSpreadStride);
        if (threadIdx.x == 0) s_tot = t;
    } else if (threadIdx.x < 2 * kWave) {
        // round r-1's totals (its slot is next cleared by round r+1)
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
        // unconditionally so rounds past the end read an empty frontier
        tot[((size_t)r2 * kSpread + threadIdx.x) * kSpreadStride] = 0ull;
        if (threadIdx.x == 0) {
            qcnt[r2] = 0;
            qover[r2] = 0;
        }
    }
    const uint32_t count = (uint32_t)(packed >> 32);
    const uint32_t edges = (uint32_t)packed;
    // vertices of nonzero degree not yet reached after round r: the number
    // reached through round r-1 was left by the previous launch
    const unsigned long long reached = reached_before + count;
    const unsigned long long unvisited = a.nnz > reached ? a.nnz - reached : 0ull;
    if (blockIdx.x == 0 && threadIdx.x == 0) a.ctl[14 + (r & 1u)] = reached;
    if (count == 0) {
        // nothing left.  The first launch to find that (round r-1 still had
        // vertices) attaches the degree-1 vertices and tells the host; the
        // launches queued behind it return at once.
        if ((s_prev >> 32) != 0) attach_leaves(a, r, q);
        return true;
    }
    const bool qvalid = qover_r == 0;
    const bool push = choose_push(a, r, count, edges, qvalid);

    uint32_t* Fs[3] = {a.F0, a.F1, a.F2};
    const uint32_t* Fc = Fs[r % 3];
    uint32_t* Fn = Fs[(r + 1) % 3];
    uint32_t* Fclr = Fs[(r + 2) % 3];
    const uint32_t* Qc = (r & 1) ? a.Q1 : a.Q0;
    const uint32_t* Pc = (r & 1) ? a.P1 : a.P0;

    const int l = lane_id();
    const int wib = threadIdx.x / kWave;
    const uint32_t gwave = blockIdx.x * kRWaves + wib;
    const uint32_t nwaves = gridDim.x * kRWaves;
    const uint32_t r1 = (r + 1) & 3u;
    QueueOut out;
    out.Q = (r & 1) ? a.Q0 : a.Q1;
    out.P = (r & 1) ? a.P0 : a.P1;
    out.qcnt = &qcnt[r1];
    out.qover = &qover[r1];
    out.qlimit = (a.force_dir == 1 || a.force_dir == 3) ? ~0ull : a.dense_thresh;
    out.tot = tot + (size_t)r1 * kSpread * kSpreadStride;

    if (blockIdx.x == 0 && threadIdx.x == 0) {
        host_store(&a.prog[0], r + 1);
        if (r < (uint32_t)kLogCap) {
            host_store(&a.log[4 * r + 0], push ? (qvalid ? 1u : 3u) : 2u);
            host_store(&a.log[4 * r + 1], count);
            host_store(&a.log[4 * r + 2], edges);
            host_store(&a.log[4 * r + 3], qvalid ? 1u : 0u);
        }
    }

    if (push) {
        // clear the bitmap that round r+1 writes
        for (int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w < a.nwords;
             w += (int64_t)gridDim.x * blockDim.x)
            Fclr[w] = 0u;
        PushPolicy pol{&a, Fc, Fn, &q, &out, r};
        if (qvalid) {
            // sparse frontier: fold U_r into V (leaves V | F_r unchanged),
            // then walk its edges in edge-balanced chunks
            for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count;
                 i += gridDim.x * blockDim.x) {
                uint32_t u = Qc[i];
                atomicOr(&a.V[u >> 5], 1u << (u & 31));
            }
            const uint32_t wc = wave_chunk(edges, nwaves, a.chunk_cap);
            const uint32_t nchunks = (edges + wc - 1) / wc;
            for (uint32_t c = gwave; c < nchunks; c += nwaves) {
                const uint32_t eb = c * wc;
                expand_range(Qc, Pc, count, edges, a.off, eb, min(edges, eb + wc), pol);
            }
        } else {
            // the frontier exists only as a bitmap (after a dense round):
            // each wavefront converts 64 words at a time to vertex ids with a
            // popcount prefix and expands them 64 at a time
            // wavefront gwave takes words gwave + nwaves * (64 * it + lane), so
            // a frontier clustered in one id range is spread over all waves
            const int64_t span = (int64_t)nwaves * 64;
            const int64_t nit = (a.nwords + span - 1) / span;
            for (int64_t it = 0; it < nit; ++it) {
                const int64_t w = gwave + (int64_t)nwaves * (64 * it + l);
                const uint32_t fw = w < a.nwords ? Fc[w] : 0u;
                if (fw) a.V[w] |= fw;
                const uint32_t c = (uint32_t)__popc(fw);
                const uint32_t inc = wave_incl_sum(c);
                const uint32_t total = __shfl(inc, 63, 64);
                const uint32_t excl = inc - c;
                for (uint32_t B = 0; B < total; B += 64) {
                    const uint32_t j = B + (uint32_t)l;
                    const bool valid = j < total;
                    int o = 0;
#pragma unroll
                    for (int s = 32; s >= 1; s >>= 1) {
                        uint32_t pv = __shfl(excl, o + s, 64);
                        if (pv <= j) o += s;
                    }
                    const uint32_t fo = __shfl(fw, o, 64);
                    const uint32_t k = j - __shfl(excl, o, 64);
                    uint32_t u = 0, dg = 0;
                    int64_t st = 0;
                    if (valid) {
                        const int64_t wo = gwave + (int64_t)nwaves * (64 * it + o);
                        u = (uint32_t)(wo * 32) + select_bit(fo, k);
                        st = a.off[u];
                        dg = a.deg[u];
                    }
                    expand_lanes(valid, u, st, dg, pol);
                }
            }
        }
        wgq_finish(q, out, true);
    } else {
        // dense round; the output is the bitmap only
        if (blockIdx.x == 0 && threadIdx.x == 0) *out.qover = 1ull;
        uint32_t found = 0, dsum = 0;
        if (2ull * unvisited >= a.nnz)
            pull_list(a, r, gwave, nwaves, Fc, Fn, Fclr, found, dsum);
        else
            pull_bitmap(a, r, gwave, nwaves, Fc, Fn, Fclr, found, dsum);
        found = wave_sum(found);
        dsum = wave_sum(dsum);
        if (l == 0 && found) {
            atomicAdd(&q.found, found);
            atomicAdd(&q.fdsum, dsum);
        }
        __syncthreads();
        if (threadIdx.x == 0 && q.found)
            atomicAdd(&out.tot[(blockIdx.x % kSpread) * kSpreadStride],
                      ((unsigned long long)q.found << 32) | q.fdsum);
    }
    return false;
}

__global__ __launch_bounds__(kRBlock, 8) void bfs_round_kernel(BfsArgs a, uint32_t r) {
    __shared__ WgQueue q;
    __shared__ unsigned long long s_tot, s_prev;
    (void)bfs_round(a, r, q, s_tot, s_prev);
}

// All rounds of one BFS in a single cooperative launch, separated by grid
// barriers (for deep graphs, where a round's work is smaller than a
// launch).  Ends when a round finds the frontier empty, or after max_rounds,
// or when a barrier is abandoned (the abort word tells the host).  One
// workgroup per CU, up to 128 VGPRs: the loop around the round keeps more
// state live, and at the 64-VGPR limit of two workgroups per CU it spilled.
__global__ __launch_bounds__(kRBlock, 4) void bfs_persistent_kernel(BfsArgs a, uint32_t* bar,
                                                                    uint32_t max_rounds) {
    __shared__ WgQueue q;
    __shared__ unsigned long long s_tot, s_prev;
    __shared__ DieInfo di;
    if (!bar_census(bar, di)) return;
    for (uint32_t r = 0; r < max_rounds; ++r) {
        if (bfs_round(a, r, q, s_tot, s_prev)) break;
        if (!grid_barrier(bar, di, r + 1)) break;
    }
}

// Kernel arguments of one BFS over workspace w (device arrays attached) with
// its progress words and round log at prog (kHostLogOff + 4 * kLogCap words).
static BfsArgs bfs_args(gbgpu_graph g, const BfsWs* w, uint32_t* prog, int32_t src,
                        int32_t* dist, int32_t* parent, const gbgpu_opts& o) {
    BfsArgs a;
    a.off = g->off;
    a.nbr = g->nbr;
    a.deg = g->deg;
    a.V = w->V;
    a.F0 = w->F[0];
    a.F1 = w->F[1];
    a.F2 = w->F[2];
    a.Q0 = w->Q[0];
    a.Q1 = w->Q[1];
    a.P0 = w->P[0];
    a.P1 = w->P[1];
    a.dist = dist;
    a.parent = (uint32_t*)parent;
    a.ctl = w->ctl;
    a.prog = prog;
    a.log = prog + kHostLogOff;
    a.head = g->head;
    a.nz = g->core;
    a.nz_head = g->core_head;
    a.nnz = g->ncore;
    a.leaf = g->leaf;
    a.nleaf = g->nleaf;
    a.src = (uint32_t)src;
    a.m32 = (uint32_t)g->m;
    a.n = g->n;
    a.nwords = g->nwords;
    a.dense_thresh = (uint64_t)g->m / (uint64_t)o.tau;
    a.stay_dense = o.beta > 0 ? (uint32_t)(g->n / o.beta) : 0xFFFFFFFFu;
    a.force_dir = o.force_direction;
    a.light = o.pull_light;
    a.chunk_cap = (uint32_t)o.wave_chunk;
    return a;
}

// Workgroups of a round launch: enough for the graph, at most o.grid.
static int bfs_round_grid(gbgpu_graph g, const gbgpu_opts& o) {
    const int64_t work = std::max<int64_t>(g->nwords / 32, g->m / 4096);
    return (int)std::min<int64_t>(std::max<int64_t>(work, 1), o.grid);
}

// Statistics of one finished BFS: bfs_stats_log adds nlog rounds of the
// round log lg (4 words per round; see gbgpu_debug_bfs_log), bfs_stats_end
// completes them from the progress words prog[0..3].
static void bfs_stats_log(gbgpu_stats* st, const volatile uint32_t* lg, size_t nlog) {
    for (size_t i = 0; i < nlog; ++i) {
        st->rounds++;
        if (lg[4 * i] == 2) st->pull_rounds++; else st->push_rounds++;
        st->reached += lg[4 * i + 1];
        st->edges_examined += lg[4 * i + 2];
    }
}

static void bfs_stats_end(gbgpu_stats* st, const uint32_t* prog, int64_t launches,
                          double kernel_ms, double wall_ms) {
    // attached degree-1 vertices: counted, and one level deeper than the
    // last round when they hang off its vertices
    st->reached += prog[2];
    st->rounds = std::max<int32_t>(st->rounds, (int32_t)prog[3] + 1);
    st->launches = (int32_t)launches;
    st->kernel_ms = kernel_ms;
    st->wall_ms = wall_ms;
}

// Whether this search runs every round in one cooperative launch (only when
// asked for: alone on the device the single launch is no faster than one
// launch per round, since a round's dependent memory trips, not the launch,
// set its time; the server asks for it on deep graphs).
static bool use_persistent(const gbgpu_opts& o) { return o.persistent > 0; }

// Runs the rounds of the search set up by bfs_init_kernel (already queued
// on `stream`) in one cooperative launch of at most `grid` workgroups (fewer
// if that many cannot all be resident), then waits for it.  *done is false
// when the launch was refused or a grid barrier gave up: the state is then
// partial and the caller runs the search again.
static int run_bfs_persistent(gbgpu_graph g, BfsWs* w, const BfsArgs& a, int grid,
                              int64_t max_rounds, hipStream_t stream, bool* done) {
    *done = false;
    int coop = 0;
    if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, g->device) !=
            hipSuccess || !coop)
        return GBGPU_OK;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, reinterpret_cast<const void*>(bfs_persistent_kernel), kRBlock, 0) !=
            hipSuccess || per_cu < 1)
        return GBGPU_OK;
    const int pgrid = std::max(1, std::min(grid, per_cu * g->num_cus));
    BfsArgs ka = a;
    uint32_t* bar = reinterpret_cast<uint32_t*>(w->ctl + kCtlWords);
    uint32_t maxr = (uint32_t)std::min<int64_t>(max_rounds, 0xFFFFFFFFll);
    void* args[] = {&ka, &bar, &maxr};
    if (hipLaunchCooperativeKernel(reinterpret_cast<const void*>(bfs_persistent_kernel),
                                   dim3(pgrid), dim3(kRBlock), args, 0, stream) != hipSuccess) {
        (void)hipGetLastError();  // refused: fall back to one launch per round
        return GBGPU_OK;
    }
    uint32_t abort_w = 0;
    GB_HIP(hipMemcpyAsync(&abort_w, bar + kBarAbort, 4, hipMemcpyDeviceToHost, stream));
    GB_HIP(hipStreamSynchronize(stream));
    *done = abort_w == 0 && w->hl.h[1] != 0;
    return GBGPU_OK;
}

// One BFS on workspace w.  The results are complete when this returns; the
// few launches queued behind the one that found the frontier empty may still
// be pending unless sync_end is set.  They only touch the workspace, and the
// next run on it (on any stream) waits for them.
int run_bfs_ws(gbgpu_graph g, BfsWs* w, int32_t src, int32_t* dist, int32_t* parent,
               const gbgpu_opts& o, gbgpu_stats* st, hipStream_t stream, bool sync_end,
               bool wait_prev) {
    const double t0 = now_ms();
    // the workspace's last user may have been another stream (not needed when
    // the previous search ran on this same stream)
    if (wait_prev) GB_HIP(hipStreamWaitEvent(stream, w->done, 0));
    const BfsArgs a = bfs_args(g, w, w->hl.d, src, dist, parent, o);
    const int grid = bfs_round_grid(g, o);
    int igrid = (int)std::min<int64_t>((g->n / 4 + kBlock - 1) / kBlock, 4096);
    if (igrid < 1) igrid = 1;
    hipLaunchKernelGGL(bfs_init_kernel, dim3(igrid), dim3(kBlock), 0, stream, a, g->pruned,
                       (uint32_t)src);
    GB_HIP(hipGetLastError());

    volatile uint32_t* hp = w->hl.h;
    hp[0] = 0;
    hp[1] = 0;
    hp[2] = 0;
    hp[3] = 0;
    if (o.profile) GB_HIP(hipEventRecord(w->ev0, stream));
    const int64_t max_rounds = std::min<int64_t>(g->n + 2, 0x7FFFFFFF);
    int64_t launches = 0;
    bool done = false;
    if (use_persistent(o)) {
        // every round in one cooperative launch; if the launch is refused or
        // a grid barrier gave up, the search runs again one launch per round
        GB_TRY(run_bfs_persistent(g, w, a, grid, max_rounds, stream, &done));
        if (done) launches = 1;
        if (!done) {
            hipLaunchKernelGGL(bfs_init_kernel, dim3(igrid), dim3(kBlock), 0, stream, a,
                               g->pruned, (uint32_t)src);
            GB_HIP(hipGetLastError());
            hp[0] = 0;
            hp[1] = 0;
            hp[2] = 0;
            hp[3] = 0;
        }
    }
    if (!done)
        GB_TRY(run_pipeline(
            hp, stream, o.rounds_per_sync, max_rounds,
            [&](int64_t r) {
                hipLaunchKernelGGL(bfs_round_kernel, dim3(grid), dim3(kRBlock), 0, stream, a,
                                   (uint32_t)r);
            },
            &launches));
    if (o.profile) GB_HIP(hipEventRecord(w->ev1, stream));
    GB_HIP(hipEventRecord(w->done, stream));
    // every round that wrote results has finished once the device reported
    // the empty frontier
    if (sync_end) GB_HIP(hipStreamSynchronize(stream));
    else if (o.profile) GB_HIP(hipEventSynchronize(w->ev1));
    const uint32_t rounds = hp[1] - 1;
    w->last_rounds = rounds;
    g->depth.store((int32_t)std::max<uint32_t>(rounds, hp[3] + 1u), std::memory_order_relaxed);
    if (st) {
        float ms = 0.f;
        if (o.profile) GB_HIP(hipEventElapsedTime(&ms, w->ev0, w->ev1));
        memset(st, 0, sizeof(*st));
        bfs_stats_log(st, hp + kHostLogOff, std::min<uint32_t>(rounds, (uint32_t)kLogCap));
        bfs_stats_end(st, (const uint32_t*)hp, launches, ms, now_ms() - t0);
    }
    return GBGPU_OK;
}

int run_bfs(gbgpu_graph g, int32_t src, int32_t* dist, int32_t* parent, const gbgpu_opts& o,
            gbgpu_stats* st, hipStream_t stream) {
    GB_TRY(ensure_bfs_ws(g));
    return run_bfs_ws(g, g->bfs, src, dist, parent, o, st, stream, false, true);
}

// k searches one after another on one stream: the next starts as soon as
// the device reports the previous one's empty frontier, without a return
// to the caller in between.
int run_bfs_many(gbgpu_graph g, const int32_t* srcs, int32_t k, int32_t* dist, int32_t* parent,
                 int64_t stride, const gbgpu_opts& o, gbgpu_stats* st, hipStream_t stream) {
    GB_TRY(ensure_bfs_ws(g));
    const double t0 = now_ms();
    gbgpu_stats sum;
    memset(&sum, 0, sizeof(sum));
    for (int32_t i = 0; i < k; ++i) {
        gbgpu_stats one;
        GB_TRY(run_bfs_ws(g, g->bfs, srcs[i], dist + (int64_t)i * stride,
                          parent + (int64_t)i * stride, o, st ? &one : nullptr, stream, false,
                          i == 0));
        if (st) {
            sum.rounds += one.rounds;
            sum.push_rounds += one.push_rounds;
            sum.pull_rounds += one.pull_rounds;
            sum.launches += one.launches;
            sum.reached += one.reached;
            sum.edges_examined += one.edges_examined;
            sum.kernel_ms += one.kernel_ms;
        }
    }
    if (st) {
        sum.wall_ms = now_ms() - t0;
        *st = sum;
    }
    return GBGPU_OK;
}

// Round log of the last BFS on this graph: 4 words per round (direction 1 =
// sparse / 2 = dense, |U_r|, sum deg(U_r), queue valid).  Used by tests and
// the benchmark's byte model.
int bfs_round_log(gbgpu_graph g, uint32_t* out, int32_t max_rounds, int32_t* nrounds) {
    if (!g->bfs) { *nrounds = 0; return GBGPU_OK; }
    const int32_t r = (int32_t)std::min<int64_t>(
        std::min<int64_t>(max_rounds, kLogCap), g->bfs->last_rounds);
    memcpy(out, g->bfs->hl.h + kHostLogOff, (size_t)r * 16);
    *nrounds = r;
    return GBGPU_OK;
}

// ---------------------------------------------------------------------------
// Allocation-free BFS (gbgpu_bfs_noalloc): the same kernels, with the
// workspace, progress words and round log in one file-scope device array
// instead of memory allocated per graph.  The host learns of the end of the
// search by copying the progress words back every few launches (there is no
// pinned memory to poll).  Launches queued past the end find an empty
// frontier and return at once, as in the pipelined driver.
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = 64ull << 20;
constexpr size_t kScratchProgBytes = (kHostLogOff + 4 * (size_t)kLogCap) * 4;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex s_scratch_mu[kMaxDevices];  // one call at a time per device
static void* s_scratch_ptr[kMaxDevices];      // device address of `scratch`, per device

size_t bfs_noalloc_ws_bytes(int64_t n, int64_t nwords) {
    return al256(kScratchProgBytes) + bfs_ws_bytes(n, nwords);
}

// Clears the progress words before the first round launch.
__global__ void bfs_prog_clear_kernel(uint32_t* prog) {
    if (threadIdx.x < 4) prog[threadIdx.x] = 0u;
}

int run_bfs_noalloc(gbgpu_graph g, int32_t src, int32_t* dist, int32_t* parent,
                    const gbgpu_opts& o, gbgpu_stats* st, hipStream_t stream) {
    const double t0 = now_ms();
    int dev = 0;
    GB_HIP(hipGetDevice(&dev));
    if (dev != g->device)
        return set_error(GBGPU_E_INVALID, "current device %d is not the graph's device %d", dev,
                         g->device);
    if (dev < 0 || dev >= kMaxDevices)
        return set_error(GBGPU_E_UNSUPPORTED, "device %d beyond the library's %d", dev,
                         kMaxDevices);
    const size_t need = bfs_noalloc_ws_bytes(g->n, g->nwords);
    if (need > kScratchBytes)
        return set_error(GBGPU_E_UNSUPPORTED,
                         "n = %lld needs %zu bytes of workspace; the allocation-free BFS "
                         "holds %zu",
                         (long long)g->n, need, kScratchBytes);
    std::lock_guard<std::mutex> lk(s_scratch_mu[dev]);
    if (!s_scratch_ptr[dev]) {
        void* ptr = nullptr;
        GB_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return set_error(GBGPU_E_HIP, "no device address for the BFS scratch array");
        s_scratch_ptr[dev] = ptr;
    }
    char* base = (char*)s_scratch_ptr[dev];
    uint32_t* prog = (uint32_t*)base;
    BfsWs w;  // device arrays only: no host log, events or owned block
    bfs_ws_attach(&w, base + al256(kScratchProgBytes), g->n, g->nwords);
    const BfsArgs a = bfs_args(g, &w, prog, src, dist, parent, o);
    const int grid = bfs_round_grid(g, o);
    int igrid = (int)std::min<int64_t>((g->n / 4 + kBlock - 1) / kBlock, 4096);
    if (igrid < 1) igrid = 1;
    hipLaunchKernelGGL(bfs_prog_clear_kernel, dim3(1), dim3(64), 0, stream, prog);
    hipLaunchKernelGGL(bfs_init_kernel, dim3(igrid), dim3(kBlock), 0, stream, a, g->pruned,
                       (uint32_t)src);
    GB_HIP(hipGetLastError());
    const int64_t max_rounds = std::min<int64_t>(g->n + 2, 0x7FFFFFFF);
    const int64_t per_check = std::max(8, o.rounds_per_sync);
    uint32_t hp[4] = {0, 0, 0, 0};
    int64_t launches = 0;
    while (launches < max_rounds) {
        const int64_t upto = std::min(max_rounds, launches + per_check);
        for (; launches < upto; ++launches)
            hipLaunchKernelGGL(bfs_round_kernel, dim3(grid), dim3(kRBlock), 0, stream, a,
                               (uint32_t)launches);
        GB_HIP(hipGetLastError());
        GB_HIP(hipMemcpyAsync(hp, prog, sizeof(hp), hipMemcpyDeviceToHost, stream));
        GB_HIP(hipStreamSynchronize(stream));
        if (hp[1]) break;
    }
    if (!hp[1])
        return set_error(GBGPU_E_HIP, "traversal did not finish within %lld launches",
                         (long long)max_rounds);
    const uint32_t rounds = hp[1] - 1;
    g->depth.store((int32_t)std::max<uint32_t>(rounds, hp[3] + 1u), std::memory_order_relaxed);
    if (st) {
        // the round log, copied back 256 rounds at a time into a stack buffer
        memset(st, 0, sizeof(*st));
        uint32_t lg[4 * 256];
        const size_t nlog = std::min<size_t>(rounds, (size_t)kLogCap);
        for (size_t i = 0; i < nlog; i += 256) {
            const size_t c = std::min<size_t>(256, nlog - i);
            GB_HIP(hipMemcpyAsync(lg, prog + kHostLogOff + 4 * i, c * 16, hipMemcpyDeviceToHost,
                                  stream));
            GB_HIP(hipStreamSynchronize(stream));
            bfs_stats_log(st, lg, c);
        }
        bfs_stats_end(st, hp, launches, 0.0, now_ms() - t0);
    }
    return GBGPU_OK;
}

}  // namespace gb
