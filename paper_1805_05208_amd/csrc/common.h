// Shared definitions for the gbgpu HIP library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <stdarg.h>

#include <algorithm>
#include <atomic>
#include <cstring>
#include <functional>
#include <mutex>
#include <string>
#include <vector>

#include "gbgpu.h"

// ---------------------------------------------------------------------------
// Host-side error reporting
// ---------------------------------------------------------------------------
namespace gb {

int set_error(int status, const char* fmt, ...);

#define GB_HIP(expr)                                                                \
    do {                                                                            \
        hipError_t _e = (expr);                                                     \
        if (_e != hipSuccess)                                                       \
            return ::gb::set_error(GBGPU_E_HIP, "%s failed: %s (%s:%d)", #expr,     \
                                   hipGetErrorString(_e), __FILE__, __LINE__);      \
    } while (0)

#define GB_TRY(expr)                       \
    do {                                   \
        int _s = (expr);                   \
        if (_s != GBGPU_OK) return _s;     \
    } while (0)

constexpr int kWave = 64;
constexpr int kBlock = 256;                 // 4 wavefronts per workgroup
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kStageCap = 256;              // per-wavefront LDS staging entries
constexpr uint32_t kNone = 0xFFFFFFFFu;

// Workspace of the single-source BFS (bfs.hip).
struct BfsWs;
// Workspace of the weighted BFS (wbfs.hip).
struct WbfsWs;
// Workspace of betweenness centrality (bc.hip).
struct BcWs;
void free_bc_ws(BcWs* w);
struct Arena;
void free_arena(Arena* a);
struct CAdj;
void free_cadj(CAdj* c);
// Workspace of multi-source BFS (multi.hip).
struct MultiWs;

}  // namespace gb

// The graph handle.  Arrays offsets / neighbors / weights are borrowed.
struct gbgpu_graph_s {
    int64_t n = 0;
    int64_t m = 0;
    const int64_t* off = nullptr;
    const int32_t* nbr = nullptr;
    const int32_t* w = nullptr;
    int32_t maxw = 0;
    int32_t minw = 1;            // smallest weight when one is below 1, else 1
    int64_t nwords = 0;          // bitmap words, padded to a multiple of 2 (64 vertices)
    uint32_t* deg = nullptr;     // owned: degree of each vertex
    uint32_t* pruned = nullptr;  // owned: bit set for vertices of degree 0 or 1 and padding
                                 // (the BFS rounds never scan them)
    uint4* head = nullptr;       // owned: first four neighbours of each vertex (kNone-padded)
    int device = 0;
    int num_cus = 256;
    std::mutex mu;               // serialises calls sharing the workspaces
    std::mutex plan_mu;          // guards the lazily built pull plan
    std::atomic<int32_t> depth{0};  // BFS depth seen by the last single-source BFS (0: none yet)
    uint4* plan = nullptr;       // owned: dense-scan work items (see ensure_pull_plan)
    uint32_t nplan = 0;
    uint32_t* core = nullptr;    // owned: ids of the vertices of degree >= 2, ascending
    uint4* core_head = nullptr;  // owned: their head records, in the same order
    uint32_t ncore = 0;
    int64_t max_degree = 0;      // set with the vertex lists
    uint2* leaf = nullptr;       // owned: (vertex, its one neighbour) for every vertex of
                                 // degree 1, ascending by vertex
    uint32_t nleaf = 0;
    gb::BfsWs* bfs = nullptr;
    gb::BfsWs* sr = nullptr;     // workspace of the Bellman-Ford / widest-path rounds
    gb::BcWs* bc = nullptr;      // workspace of betweenness centrality
    gb::Arena* cc = nullptr;     // device arena of the LDD / connectivity calls
    gb::CAdj* cadj = nullptr;    // compressed copy of the lists and its BFS workspace
    gb::WbfsWs* wbfs = nullptr;
    gb::MultiWs* multi = nullptr;
    // owned, built on the first weighted BFS: every list re-ordered by
    // (weight, neighbour), neighbours and 16-bit weights (dense weighted
    // steps stop at the first in-bucket neighbour in that order)
    uint32_t* wsort_nbr = nullptr;
    uint16_t* wsort_w = nullptr;
    std::mutex wsort_mu;
};

namespace gb {
// One BFS query of a batch: graph, source, output rows.
struct MsQuery {
    gbgpu_graph g;
    int32_t src;
    int32_t* dist;
    int32_t* parent;
};

// Round-boundary admission into a running single-group batch: called with
// the next round r, the number of free source slots and whether the group
// has run out of work (it ends unless someone joins); appends the queries
// that join the group before round r.
using MsJoinHook =
    std::function<void(uint32_t r, int room, bool idle, std::vector<MsQuery>* add)>;

void free_bfs_ws(BfsWs* w);
void free_wbfs_ws(WbfsWs* w);
void free_multi_ws(MultiWs* w);
double now_ms();
int64_t now_ns();
gbgpu_opts resolve_opts(const gbgpu_opts* o);
// Index of the reserved option word resolve_opts sets to 1 when the caller
// left tau at 0 (the library's default).
constexpr int kTauDefaulted = 0;
int ensure_pull_plan(gbgpu_graph g);
constexpr uint32_t kPlanCap = 1024;   // max edges of one dense-scan work item
constexpr uint32_t kPlanHub = 0xFFFFFFFFu;
// The server packs BFS queries only on graphs a search has shown to be at
// most this deep: a packed group holds every query in it until its last
// round, so on a long diameter the packed queries wait far longer than
// queries run one at a time (batched calls on such graphs still pay off:
// 64 sources on the 256^3 torus, 408 ms against 684 one at a time).
constexpr int32_t kDeepGraph = 64;

// Words of coherent pinned host memory that the traversal kernels write with
// system-scope stores and the host reads directly (no copy commands): the
// progress words of a launch pipeline and the per-step log.
//   [0] number of launches that have started
//   [1] 1 + index of the launch that found nothing left to do (0 before)
//   [2] overflow flag (weighted BFS buckets)
//   [kHostLogOff ...] 4 words per step
struct HostLog {
    uint32_t* h = nullptr;  // host address
    uint32_t* d = nullptr;  // device address of the same memory
};
constexpr size_t kHostLogOff = 16;

// Workspace of the frontier-round traversals (BFS rounds in bfs.hip; the
// Bellman-Ford / widest-path rounds in sr.hip use one of their own).
constexpr int kLogCap = 8192;  // rounds kept in the pinned round log
struct BfsWs {
    int64_t n = 0;
    int64_t nwords = 0;
    uint32_t* V = nullptr;
    uint32_t* F[3] = {nullptr, nullptr, nullptr};
    uint32_t* Q[2] = {nullptr, nullptr};
    uint32_t* P[2] = {nullptr, nullptr};
    unsigned long long* ctl = nullptr;  // qcnt[4], qover[4] at +4/+8, end reported at +12,
                                        // reached counts at +14/+15, totals at +64
    HostLog hl;                         // progress words + round log (host memory)
    uint32_t last_rounds = 0;           // rounds of the last run on this workspace
    void* block = nullptr;              // owned device block (NULL when borrowed)
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    hipEvent_t done = nullptr;          // after the last launch of the last run
};
int host_log_alloc(HostLog* hl, size_t log_steps);
void host_log_free(HostLog* hl);

// Issues launch(0), launch(1), ... on `stream`, keeping `ahead` launches
// queued beyond the last one the device has reported as started, until a
// launch reports that nothing is left (prog[1] != 0).  *issued receives the
// number of launches issued.  Fails if max_launches would be exceeded or the
// stream reports an error.
int run_pipeline(volatile uint32_t* prog, hipStream_t stream, int ahead, int64_t max_launches,
                 const std::function<void(int64_t)>& launch, int64_t* issued);
}  // namespace gb

// ---------------------------------------------------------------------------
// Device helpers (wave64)
// ---------------------------------------------------------------------------
namespace gb {

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// Number of set bits of `mask` in lanes below this one.
__device__ __forceinline__ uint32_t mbcnt(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ int first_lane(uint64_t mask) { return __ffsll((long long)mask) - 1; }
__device__ __forceinline__ int last_lane(uint64_t mask) { return 63 - __clzll((long long)mask); }

// Store into coherent host memory, visible to the host without a copy.
__device__ __forceinline__ void host_store(uint32_t* p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Orders this wavefront's LDS writes before its later LDS reads.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint32_t wave_incl_sum(uint32_t x) {
    const int l = lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t y = __shfl_up(x, d, 64);
        if (l >= d) x += y;
    }
    return x;
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t x) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
    return x;
}

__device__ __forceinline__ uint64_t shfl64(uint64_t x, int src) {
    uint32_t lo = __shfl((uint32_t)x, src, 64);
    uint32_t hi = __shfl((uint32_t)(x >> 32), src, 64);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ bool test_bit(const uint32_t* bm, uint32_t v) {
    return (bm[v >> 5] >> (v & 31)) & 1u;
}

// Largest i in [0, cnt) with P[i] <= x, where P is non-decreasing and
// P[0] <= x.  A 64-ary search: every step probes 64 evenly spaced entries.
__device__ __forceinline__ uint32_t wave_search(const uint32_t* __restrict__ P, uint32_t cnt,
                                                uint32_t x) {
    const int l = lane_id();
    uint32_t lo = 0, hi = cnt;
    while (hi - lo > 64) {
        uint32_t stride = (hi - lo + 63) / 64;
        uint32_t i = lo + (uint32_t)l * stride;
        bool ok = i < hi && P[i] <= x;
        uint64_t b = ballot(ok);
        uint32_t L = (uint32_t)last_lane(b);
        lo = lo + L * stride;
        hi = min(hi, lo + stride);
    }
    uint32_t i = lo + (uint32_t)l;
    bool ok = i < hi && P[i] <= x;
    return lo + (uint32_t)last_lane(ballot(ok));
}

// Edge-balanced expansion of a frontier held as (Q, P): Q[i] is a vertex and
// P[i] the exclusive prefix sum of the degrees of Q[0..i-1]; the frontier's
// edges form one index space [0, E).  The calling wavefront walks edge range
// [e_begin, e_end) 64 edges at a time (the logical blocks of the paper's
// edgeMapBlocked, which may split one high-degree vertex over many workers),
// loading 64 frontier entries at once and finding each lane's entry with a
// six-step shuffle search.  Policy provides:
//   uint32_t aux(uint32_t u)             per-entry value (e.g. a stale flag)
//   void edge(bool act, uint32_t u, uint32_t aux, int64_t e, bool first)
//                                        first: e is u's first edge (exactly
//                                        one lane over the whole range sees it)
//   void window_done()                   after each window of <= 64 edges
//   static constexpr bool kSkipDead      skip edge ranges of entries whose
//                                        aux() is 0 without visiting them
// edge() and window_done() are called by all 64 lanes together (act = lane
// has an edge).
template <typename Policy>
__device__ __forceinline__ void expand_range(const uint32_t* __restrict__ Q,
                                             const uint32_t* __restrict__ P, uint32_t cnt,
                                             uint32_t E, const int64_t* __restrict__ off,
                                             uint32_t e_begin, uint32_t e_end, Policy& pol) {
    const int l = lane_id();
    uint32_t base = wave_search(P, cnt, e_begin);
    uint32_t myP, myU, myA, endLoaded;
    int64_t myS;
    uint64_t live = 0;
    auto load = [&](uint32_t b) {
        uint32_t i = b + (uint32_t)l;
        bool ok = i < cnt;
        myP = ok ? P[i] : 0xFFFFFFFFu;
        myU = ok ? Q[i] : 0u;
        myS = ok ? off[myU] : 0;
        myA = ok ? pol.aux(myU) : 0u;
        endLoaded = (b + 64 < cnt) ? P[b + 64] : E;
        live = ballot(ok && myA != 0u);
    };
    // owner among the loaded entries: largest lane with P <= x
    auto owner = [&](uint32_t x) {
        int o = 0;
#pragma unroll
        for (int s = 32; s >= 1; s >>= 1) {
            uint32_t pv = __shfl(myP, o + s, 64);
            if (pv <= x) o += s;
        }
        return o;
    };
    load(base);
    uint32_t e = e_begin;
    while (e < e_end) {
        if (e >= endLoaded) {
            base += 64;
            load(base);
            continue;
        }
        if (Policy::kSkipDead) {
            // jump over edge ranges of entries the policy marks dead
            const int oe = owner(e);  // wave-uniform
            if (!((live >> oe) & 1ull)) {
                const uint64_t after = oe == 63 ? 0ull : (live & (~0ull << (oe + 1)));
                if (after == 0) {
                    e = endLoaded;
                } else {
                    e = max(e, __shfl(myP, first_lane(after), 64));
                }
                continue;
            }
        }
        const uint32_t lim = min(e_end, endLoaded);
        const uint32_t t = e + (uint32_t)l;
        const bool act = t < lim;
        const int o = owner(t);
        const uint32_t u = __shfl(myU, o, 64);
        const uint32_t a = __shfl(myA, o, 64);
        const int64_t s0 = (int64_t)shfl64((uint64_t)myS, o);
        const uint32_t p0 = __shfl(myP, o, 64);
        pol.edge(act, u, a, s0 + (int64_t)(t - p0), act && t == p0);
        pol.window_done();
        e = min(e + 64u, lim);
        if (e < e_end && e < endLoaded && (uint64_t)e + 63u >= endLoaded) {
            // the next window runs past the loaded entries: reload starting at
            // the entry that owns edge e
            const int o2 = owner(e);
            if (o2 > 0) {
                base += (uint32_t)o2;
                load(base);
            }
        }
    }
}

// Expansion of up to 64 frontier entries held in lanes (vertex u, list start,
// degree): their edges are concatenated and walked 64 at a time with the same
// shuffle search as expand_range; aux is a per-entry value handed to edge()
// like the one expand_range takes from the policy.  Lanes that are not valid, or have degree
// 0, may sit anywhere: their prefix equals the next lane's, and the search
// returns the largest lane whose prefix is <= the edge index, which always
// owns edges.  Wave-uniform.
template <typename Policy>
__device__ __forceinline__ void expand_lanes(bool valid, uint32_t u, int64_t start, uint32_t deg,
                                             Policy& pol, uint32_t aux = 1u) {
    const int l = lane_id();
    const uint32_t d = valid ? deg : 0u;
    const uint32_t inc = wave_incl_sum(d);
    const uint32_t T = __shfl(inc, 63, 64);
    const uint32_t myP = inc - d;
    for (uint32_t e = 0; e < T; e += 64) {
        const uint32_t t = e + (uint32_t)l;
        const bool act = t < T;
        int o = 0;
#pragma unroll
        for (int s = 32; s >= 1; s >>= 1) {
            uint32_t pv = __shfl(myP, o + s, 64);
            if (pv <= t) o += s;
        }
        const uint32_t uo = __shfl(u, o, 64);
        const int64_t so = (int64_t)shfl64((uint64_t)start, o);
        const uint32_t po = __shfl(myP, o, 64);
        pol.edge(act, uo, __shfl(aux, o, 64), so + (int64_t)(t - po), act && t == po);
        pol.window_done();
    }
}

// Index of the k-th set bit (k < popcount(x)) of x.
__device__ __forceinline__ uint32_t select_bit(uint32_t x, uint32_t k) {
    uint32_t pos = 0;
#pragma unroll
    for (int w = 16; w >= 1; w >>= 1) {
        const uint32_t lowc = (uint32_t)__popc(x & ((1u << w) - 1u));
        if (k >= lowc) {
            k -= lowc;
            x >>= w;
            pos += (uint32_t)w;
        }
    }
    return pos;
}

// Edge chunk size for one wavefront: enough to give every wavefront of the
// grid work when the frontier is small, at most `cap` edges.
__device__ __forceinline__ uint32_t wave_chunk(uint32_t E, uint32_t nwaves, uint32_t cap) {
    uint32_t c = (E + nwaves - 1) / nwaves;
    c = (c + 63u) & ~63u;
    if (c < 64u) c = 64u;
    if (c > cap) c = cap;
    return c;
}

}  // namespace gb
