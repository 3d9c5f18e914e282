// Integral-weight SSSP (weighted BFS) with distance buckets.
//
// Method (paper: wBFS algorithm box, after Julienne): buckets hold vertices
// by tentative distance; nextBucket returns the smallest non-empty bucket b;
// edgeMapData relaxes the edges of bucket b's vertices with a priority-write
// (writeMin) of the new distance; vertices whose distance dropped are moved to
// their new bucket (vertexMap Reset + updateBuckets).  Because weights are at
// least 1, every vertex in bucket b is settled when b is extracted, so each
// vertex's edges are relaxed exactly once (O(m) work).
//
// GPU form:
//   key[v]   uint64 = (distance << 32) | parent.  One 64-bit atomicMin is the
//            priority-write; it also keeps the smallest parent among the
//            neighbours that reach v at its final distance, so
//            parent[v] = min{u in N(v) : D[u] + w(u,v) = D[v]} without a
//            separate pass.
//   buckets  a ring of NB slots (NB a power of two, NB >= 2*maxw + 1), slot
//            b mod NB holding bucket b.  Pending distances lie in
//            (b, b + maxw] while bucket b is processed, so the ring never
//            wraps onto a live bucket, and the slot of the previous bucket can
//            be reset by the next step without racing its writers.
//            Each slot stores vertex ids Q and the exclusive prefix sum P of
//            their degrees (for edge-balanced expansion) behind one packed
//            counter (count << 32 | sum of degrees).
//   moves    a relaxation that lowers D[v] appends v to the bucket of the new
//            distance; an entry whose vertex has since moved lower is stale
//            and is skipped when its bucket is extracted (GetBucketNum reads
//            the current distance).  So updateBuckets is fused into the
//            relaxation and each (vertex, distance) pair is appended at most
//            once.
//   steps    one kernel launch per bucket: the launch finds b itself (the
//            smallest non-empty slot after the previous bucket), resets the
//            previous slot, and relaxes bucket b.  The host only checks a done
//            flag every few hundred launches.
//   dense    edgeMapData's dense form for a heavy bucket (entries + their
//            degrees > m / tau): the launch that finds b only marks b's live
//            vertices in a bucket bitmap (and the settled bitmap); the next
//            launch pulls: every unsettled vertex v takes min over u in bucket
//            b of ((b + w(u,v)) << 32 | u), which is the same value the pushes
//            of bucket b would leave in key[v].  The pull reads a copy of each
//            list ordered by (weight, neighbour), built once per graph, so the
//            first in-bucket neighbour in that order is the minimum and the
//            scan stops there, or at the first weight too large to lower
//            key[v].  The handover between the two launches goes through
//            control words on the device, so the host still launches blindly.

#include <rocprim/device/device_segmented_radix_sort.hpp>

#include "common.h"
#include "emit.h"

namespace gb {

constexpr int kWLogCap = 16384;
constexpr int kWbfsTau = 10;  // default dense threshold m / 10 (see run_wbfs_ws)
constexpr uint32_t kStart = 0xFFFFFFFFu;  // "bucket before 0"
constexpr uint32_t kDone = 0xFFFFFFFEu;

struct WbfsWs {
    int64_t n = 0;
    uint32_t NB = 0;
    uint32_t C = 0;
    unsigned long long* key = nullptr;
    uint32_t* Qs = nullptr;
    uint32_t* Ps = nullptr;
    unsigned long long* sc = nullptr;
    uint32_t* S = nullptr;     // settled bitmap
    uint32_t* Fb = nullptr;    // two bucket bitmaps for dense steps
    uint32_t* ctl = nullptr;   // [0..1] bucket of step j (j & 1), [2] done, [3] overflow,
                               // [4..5] step state left by launch j (j & 1)
    HostLog hl;                // progress words + step log (host memory)
    uint32_t last_steps = 0;   // step launches of the last run on this workspace
    void* block = nullptr;     // owned device block (NULL when borrowed)
    size_t bytes = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
};

void free_wbfs_ws(WbfsWs* w) {
    if (!w) return;
    if (w->block) (void)hipFree(w->block);
    host_log_free(&w->hl);
    if (w->ev0) (void)hipEventDestroy(w->ev0);
    if (w->ev1) (void)hipEventDestroy(w->ev1);
    delete w;
}

uint32_t wbfs_window(int32_t maxw, int32_t req) {
    uint32_t need = 2u * (uint32_t)std::max(maxw, 1) + 1u;
    uint32_t nb = 2;
    while (nb < need) nb <<= 1;
    if (req > 0) {
        uint32_t r = 2;
        while (r < (uint32_t)req) r <<= 1;
        nb = std::max(nb, r);
    }
    return nb;
}

uint32_t wbfs_default_capacity(int64_t n) {
    return (uint32_t)std::min<int64_t>(n, std::max<int64_t>(4096, n / 4));
}

static size_t wal(size_t x) { return (x + 255) & ~(size_t)255; }

size_t wbfs_bytes(int64_t n, uint32_t NB, uint32_t C) {
    return wal((size_t)n * 8) + 2 * wal((size_t)NB * C * 4) +
           wal((size_t)NB * 8 * kSpreadStride) + wal(64) + 3 * wal((size_t)((n + 63) / 64) * 8);
}

void wbfs_ws_attach(WbfsWs* w, void* mem, int64_t n, uint32_t NB, uint32_t C) {
    w->n = n;
    w->NB = NB;
    w->C = C;
    w->bytes = wbfs_bytes(n, NB, C);
    char* p = (char*)mem;
    w->key = (unsigned long long*)p; p += wal((size_t)n * 8);
    w->Qs = (uint32_t*)p; p += wal((size_t)NB * C * 4);
    w->Ps = (uint32_t*)p; p += wal((size_t)NB * C * 4);
    w->sc = (unsigned long long*)p; p += wal((size_t)NB * 8 * kSpreadStride);
    w->ctl = (uint32_t*)p; p += wal(64);
    w->S = (uint32_t*)p; p += wal((size_t)((n + 63) / 64) * 8);
    w->Fb = (uint32_t*)p;  // two bitmaps of (n + 63) / 64 * 2 words, each 256-aligned
}

int wbfs_ws_host_init(WbfsWs* w) {
    GB_TRY(host_log_alloc(&w->hl, kWLogCap));
    if (hipEventCreate(&w->ev0) != hipSuccess || hipEventCreate(&w->ev1) != hipSuccess)
        return set_error(GBGPU_E_HIP, "wBFS workspace: event creation failed");
    return GBGPU_OK;
}

WbfsWs* wbfs_ws_new() { return new WbfsWs(); }

static int ensure_wbfs_ws(gbgpu_graph g, uint32_t NB, uint32_t C) {
    if (g->wbfs && g->wbfs->NB == NB && g->wbfs->C == C) return GBGPU_OK;
    free_wbfs_ws(g->wbfs);
    g->wbfs = nullptr;
    WbfsWs* w = new WbfsWs();
    const size_t bytes = wbfs_bytes(g->n, NB, C);
    hipError_t e = hipMalloc(&w->block, bytes);
    if (e != hipSuccess) {
        delete w;
        return set_error(GBGPU_E_NOMEM, "wBFS workspace of %zu bytes: %s", bytes,
                         hipGetErrorString(e));
    }
    wbfs_ws_attach(w, w->block, g->n, NB, C);
    int s = wbfs_ws_host_init(w);
    if (s != GBGPU_OK) {
        free_wbfs_ws(w);
        return s;
    }
    g->wbfs = w;
    return GBGPU_OK;
}

// ---------------------------------------------------------------------------
// Lists ordered by (weight, neighbour), for the dense steps: a stable
// segmented radix sort of each list (already ascending by neighbour) by its
// 11-bit weights.  Built once per graph by the first weighted BFS; 6 bytes
// per stored edge.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void wsort_keys_kernel(const int32_t* wt, int64_t m,
                                                           uint16_t* k) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = tid; i < m; i += stride) k[i] = (uint16_t)wt[i];
}

static int ensure_wsort(gbgpu_graph g, hipStream_t stream) {
    std::lock_guard<std::mutex> lk(g->wsort_mu);
    if (g->wsort_nbr) return GBGPU_OK;
    const size_t m = (size_t)std::max<int64_t>(g->m, 1);
    uint16_t* kin = nullptr;
    uint16_t* kout = nullptr;
    uint32_t* vout = nullptr;
    void* tmp = nullptr;
    auto fail = [&](int st) {
        if (kin) (void)hipFree(kin);
        if (kout) (void)hipFree(kout);
        if (vout) (void)hipFree(vout);
        if (tmp) (void)hipFree(tmp);
        return st;
    };
    if (hipMalloc(&kin, m * 2) != hipSuccess || hipMalloc(&kout, m * 2) != hipSuccess ||
        hipMalloc(&vout, m * 4) != hipSuccess)
        return fail(set_error(GBGPU_E_NOMEM, "weight-ordered lists: %zu bytes", m * 8));
    if (g->m > 0) {
        const int grid = (int)std::min<int64_t>((g->m + kBlock - 1) / kBlock, 8192);
        hipLaunchKernelGGL(wsort_keys_kernel, dim3(grid), dim3(kBlock), 0, stream, g->w, g->m,
                           kin);
        if (hipGetLastError() != hipSuccess)
            return fail(set_error(GBGPU_E_HIP, "weight key kernel failed"));
        const uint32_t* vin = reinterpret_cast<const uint32_t*>(g->nbr);
        size_t tb = 0;
        if (rocprim::segmented_radix_sort_pairs(nullptr, tb, kin, kout, vin, vout,
                                                (unsigned int)g->m, (unsigned int)g->n, g->off,
                                                g->off + 1, 0u, 11u, stream) != hipSuccess)
            return fail(set_error(GBGPU_E_HIP, "weight-ordered lists: sort sizing failed"));
        if (hipMalloc(&tmp, std::max<size_t>(tb, 1)) != hipSuccess)
            return fail(set_error(GBGPU_E_NOMEM, "weight-ordered lists: sort storage"));
        if (rocprim::segmented_radix_sort_pairs(tmp, tb, kin, kout, vin, vout,
                                                (unsigned int)g->m, (unsigned int)g->n, g->off,
                                                g->off + 1, 0u, 11u, stream) != hipSuccess ||
            hipStreamSynchronize(stream) != hipSuccess)
            return fail(set_error(GBGPU_E_HIP, "weight-ordered lists: sort failed"));
    }
    (void)hipFree(kin);
    if (tmp) (void)hipFree(tmp);
    g->wsort_w = kout;
    g->wsort_nbr = vout;
    return GBGPU_OK;
}

struct WbfsArgs {
    const int64_t* off;
    const int32_t* nbr;
    const int32_t* wt;
    const uint32_t* snbr;    // lists ordered by (weight, neighbour): neighbours
    const uint16_t* sw;      // ... and their weights
    const uint32_t* deg;
    unsigned long long* key;
    uint32_t* Qs;
    uint32_t* Ps;
    unsigned long long* sc;
    uint32_t* S;
    uint32_t* Fb;            // bucket bitmap p at Fb + p * fb_stride
    uint32_t* ctl;
    uint32_t* prog;          // host progress words (device address)
    uint32_t* log;           // host step log (device address)
    const uint4* plan;       // dense-scan work items (runs and hub pieces)
    int64_t n;
    uint32_t NB;
    uint32_t C;
    uint32_t chunk_cap;
    uint32_t nw32;           // words of one bitmap that cover n vertices
    uint32_t fb_stride;
    uint32_t nplan;
    uint32_t dense_mode;     // 0 by threshold, 1 never, 2 always, 3 odd buckets
    unsigned long long dense_thresh;
};

// Step state a launch leaves for the next one (ctl[4 + (j & 1)]).
constexpr uint32_t kStPull = 1u;      // next launch pulls bucket ctl[j & 1] ...
constexpr uint32_t kStPullPar = 2u;   // ... with bucket bitmap 1 (else 0)
constexpr uint32_t kStClear = 4u;     // next launch zeroes a bucket bitmap ...
constexpr uint32_t kStClearPar = 8u;  // ... bitmap 1 (else 0)
constexpr uint32_t kStNextPar = 16u;  // the next dense step uses bitmap 1 (else 0)

// Step kinds recorded in the log.
constexpr uint32_t kModePush = 0u, kModeMark = 1u, kModePull = 2u;

__global__ __launch_bounds__(kBlock) void wbfs_init_kernel(WbfsArgs a, uint32_t src) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = tid; v < a.n; v += stride) a.key[v] = v == src ? (unsigned long long)src : ~0ull;
    for (int64_t i = tid; i < (a.n + 31) / 32; i += stride) {
        a.S[i] = 0u;
        a.Fb[i] = 0u;
        a.Fb[a.fb_stride + i] = 0u;
    }
    for (int64_t i = tid; i < a.NB; i += stride)
        a.sc[i * kSpreadStride] = i == 0 ? ((1ull << 32) | a.deg[src]) : 0ull;
    if (tid == 0) {
        a.Qs[0] = src;
        a.Ps[0] = 0;
        a.ctl[0] = 0;
        a.ctl[1] = kStart;
        a.ctl[2] = 0;
        a.ctl[3] = 0;
        a.ctl[4] = 0;
        a.ctl[5] = 0;
    }
}

// Workgroup staging of moved vertices: (vertex, new distance).  At the end of
// the launch they are grouped by target bucket with a counting sort in LDS,
// each non-empty target gets ONE packed reservation per workgroup, and a
// workgroup scan produces the degree prefix sums within each target.
constexpr int kMaxLdsNB = 256;
constexpr int kWgCapW = 4096;  // LDS entries per workgroup (two workgroups per CU)

struct WgBuckets {
    uint32_t v[kWgCapW];
    uint32_t d[kWgCapW];
    uint32_t sv[kWgCapW];
    uint32_t sdeg[kWgCapW];
    uint32_t hcnt[kMaxLdsNB];
    uint32_t hdeg[kMaxLdsNB];
    uint32_t hoff[kMaxLdsNB + 1];
    uint32_t hcur[kMaxLdsNB];
    unsigned long long hbase[kMaxLdsNB];
    uint32_t cnt;
    uint32_t wsum[kRWaves];
};

__device__ __forceinline__ unsigned long long* slot_counter(const WbfsArgs& a, uint32_t t) {
    return a.sc + (size_t)t * kSpreadStride;
}

// Wave-level fallback: lanes with the same target share one reservation.
__device__ __forceinline__ void wave_bucket_emit(bool take, uint32_t v, uint32_t nd,
                                                 const WbfsArgs& a) {
    const int l = lane_id();
    const uint32_t dv = take ? a.deg[v] : 0u;
    const uint32_t t = nd & (a.NB - 1);
    uint64_t pend = ballot(take);
    while (pend) {
        const int ld = first_lane(pend);
        const uint32_t tt = __shfl(t, ld, 64);
        const bool mine = take && t == tt;
        const uint64_t mk = ballot(mine);
        const uint32_t x = mine ? dv : 0u;
        const uint32_t inc = wave_incl_sum(x);
        const uint32_t tot = __shfl(inc, 63, 64);
        unsigned long long packed = 0;
        if (l == ld)
            packed = atomicAdd(slot_counter(a, tt), ((unsigned long long)__popcll(mk) << 32) | tot);
        packed = shfl64(packed, ld);
        if (mine) {
            const uint32_t pos = (uint32_t)(packed >> 32) + mbcnt(mk);
            if (pos < a.C) {
                a.Qs[(size_t)tt * a.C + pos] = v;
                a.Ps[(size_t)tt * a.C + pos] = (uint32_t)packed + inc - x;
            } else {
                a.ctl[3] = 1u;
            }
        }
        pend &= ~mk;
    }
}

__device__ __forceinline__ void wgb_push(WgBuckets& q, bool take, uint32_t v, uint32_t nd,
                                         const WbfsArgs& a) {
    const uint64_t m = ballot(take);
    if (!m) return;
    const int l = lane_id();
    const uint32_t k = (uint32_t)__popcll(m);
    const int ld = first_lane(m);
    uint32_t pos0 = kNone;
    if (l == ld && a.NB <= (uint32_t)kMaxLdsNB) {
        uint32_t old = *(volatile uint32_t*)&q.cnt;
        for (;;) {
            if (old + k > (uint32_t)kWgCapW) break;
            uint32_t prev = atomicCAS(&q.cnt, old, old + k);
            if (prev == old) {
                pos0 = old;
                break;
            }
            old = prev;
        }
    }
    pos0 = __shfl(pos0, ld, 64);
    if (pos0 != kNone) {
        if (take) {
            const uint32_t i = pos0 + mbcnt(m);
            q.v[i] = v;
            q.d[i] = nd;
        }
    } else {
        wave_bucket_emit(take, v, nd, a);
    }
}

// Workgroup-uniform: moves the buffered entries to their buckets and empties
// the buffer.
__device__ __forceinline__ void wgb_flush(WgBuckets& q, const WbfsArgs& a) {
    __syncthreads();
    const uint32_t n = q.cnt;
    __syncthreads();  // every thread has read n before anyone can append again
    if (n == 0) return;  // workgroup-uniform
    const int t = threadIdx.x;
    const int nt = blockDim.x;
    const uint32_t NB = a.NB;
    const uint32_t mask = NB - 1;
    for (int i = t; i < (int)NB; i += nt) {
        q.hcnt[i] = 0;
        q.hdeg[i] = 0;
    }
    __syncthreads();
    for (uint32_t i = t; i < n; i += nt) {
        const uint32_t tt = q.d[i] & mask;
        atomicAdd(&q.hcnt[tt], 1u);
        atomicAdd(&q.hdeg[tt], a.deg[q.v[i]]);
    }
    __syncthreads();
    if (t < kWave) {
        // exclusive scan of the per-target counts (NB <= 256)
        uint32_t carry = 0;
        for (uint32_t b0 = 0; b0 < NB; b0 += 64) {
            const uint32_t i = b0 + (uint32_t)t;
            const uint32_t x = i < NB ? q.hcnt[i] : 0u;
            const uint32_t inc = wave_incl_sum(x);
            if (i < NB) {
                q.hoff[i] = carry + inc - x;
                q.hcur[i] = carry + inc - x;
            }
            carry += __shfl(inc, 63, 64);
        }
        if (t == 0) q.hoff[NB] = carry;
    }
    for (int i = t; i < (int)NB; i += nt) {
        const uint32_t c = q.hcnt[i];
        unsigned long long packed = 0;
        if (c) packed = atomicAdd(slot_counter(a, (uint32_t)i), ((unsigned long long)c << 32) | q.hdeg[i]);
        q.hbase[i] = packed;
    }
    __syncthreads();
    for (uint32_t i = t; i < n; i += nt) {
        const uint32_t tt = q.d[i] & mask;
        const uint32_t pos = atomicAdd(&q.hcur[tt], 1u);
        const uint32_t v = q.v[i];
        q.sv[pos] = v;
        q.sdeg[pos] = a.deg[v];
    }
    __syncthreads();
    // workgroup exclusive scan over sdeg[0..n); result into q.v (free now)
    constexpr int PER = kWgCapW / kRBlock;
    const int l = lane_id();
    const int wv = t / kWave;
    uint32_t loc[PER];
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const uint32_t idx = (uint32_t)(PER * t + i);
        const uint32_t x = idx < n ? q.sdeg[idx] : 0u;
        loc[i] = s;
        s += x;
    }
    const uint32_t inc = wave_incl_sum(s);
    if (l == 63) q.wsum[wv] = inc;
    __syncthreads();
    if (t < kWave) {
        const uint32_t x = t < kRWaves ? q.wsum[t] : 0u;
        const uint32_t c = wave_incl_sum(x);
        if (t < kRWaves) q.wsum[t] = c - x;
    }
    __syncthreads();
    const uint32_t off = q.wsum[wv] + inc - s;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const uint32_t idx = (uint32_t)(PER * t + i);
        if (idx < n) q.v[idx] = off + loc[i];
    }
    __syncthreads();
    // find the target of this thread's first position, then walk forward
    const uint32_t p0 = (uint32_t)(PER * t);
    if (p0 < n) {
        uint32_t lo = 0, hi = NB;  // largest tt with hoff[tt] <= p0
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (q.hoff[mid] <= p0) lo = mid; else hi = mid;
        }
        uint32_t tt = lo;
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const uint32_t idx = p0 + (uint32_t)i;
            if (idx >= n) break;
            while (q.hoff[tt + 1] <= idx) ++tt;
            const uint32_t seg = q.hoff[tt];
            const unsigned long long hb = q.hbase[tt];
            const uint32_t pos = (uint32_t)(hb >> 32) + (idx - seg);
            if (pos < a.C) {
                a.Qs[(size_t)tt * a.C + pos] = q.sv[idx];
                a.Ps[(size_t)tt * a.C + pos] = (uint32_t)hb + q.v[idx] - q.v[seg];
            } else {
                a.ctl[3] = 1u;
            }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) q.cnt = 0;
    __syncthreads();
}

// Workgroup-uniform: flush when fewer than `room` free entries remain.
__device__ __forceinline__ void wgb_maybe_flush(WgBuckets& q, const WbfsArgs& a, uint32_t room) {
    __syncthreads();
    const uint32_t n = q.cnt;
    __syncthreads();
    if (n + room > (uint32_t)kWgCapW) wgb_flush(q, a);
}

struct RelaxPolicy {
    const WbfsArgs* a;
    WgBuckets* q;
    uint32_t b;
    static constexpr bool kSkipDead = true;

    // entry u of bucket b is live iff its current distance is still b
    __device__ __forceinline__ uint32_t aux(uint32_t u) const {
        return (uint32_t)(a->key[u] >> 32) == b ? 1u : 0u;
    }

    // A live entry is settled (weights >= 1).  The lane that relaxes its first
    // edge records that in the settled bitmap, once per vertex, so that later
    // relaxations towards it skip the random key read.  Vertices without
    // edges are never relaxation targets and need no bit.
    __device__ __forceinline__ void edge(bool act, uint32_t u, uint32_t live, int64_t e,
                                         bool first) {
        bool moved = false;
        uint32_t v = 0, nd = 0;
        if (first && live) atomicOr(&a->S[u >> 5], 1u << (u & 31));
        if (act && live) {
            v = (uint32_t)a->nbr[e];
            nd = b + (uint32_t)a->wt[e];
            const unsigned long long nk = ((unsigned long long)nd << 32) | u;
            if (!test_bit(a->S, v) && nk < a->key[v]) {
                const unsigned long long old = atomicMin(&a->key[v], nk);
                moved = nd < (uint32_t)(old >> 32);
            }
        }
        wgb_push(*q, moved, v, nd, *a);
    }

    __device__ __forceinline__ void window_done() {}
};

constexpr int kPullWin = 2;  // 64-edge windows whose loads are issued together

// One dense-scan work item: a run of at most 64 consecutive vertices whose
// lists hold at most 1024 edges together, or a piece of at most 1024 edges of
// one high-degree vertex.  Settled vertices are skipped.  Wave-uniform.
//
// The lists are read in (weight, neighbour) order.  A candidate from an
// in-bucket neighbour u is ((b + w(u,v)) << 32 | u), so in that order the
// first in-bucket neighbour gives the minimum and the scan of v ends there;
// it also ends at the first weight above room = d(v) - b, the largest weight
// that can still lower key[v] (an equal distance can still bring a smaller
// parent).
// A run's per-vertex minimum slot holds ~0 (scan going on, nothing found),
// a candidate key, or kScanEnded (ended by a heavy edge without a candidate;
// every real key is smaller, since distances stay below 2^32 - 2).
constexpr unsigned long long kScanEnded = ~0ull - 1ull;

__device__ __forceinline__ void wbfs_pull_item(const WbfsArgs& a, const uint32_t* F, uint32_t b,
                                               uint4 it, unsigned long long* smin,
                                               WgBuckets& q) {
    const int l = lane_id();
    bool moved = false;
    uint32_t v = 0, nd = 0;
    if (it.z == kPlanHub) {
        v = it.x + (uint32_t)l;
        // the settled bit, degree, list start and key are loaded together
        // (one trip; the run's vertices are consecutive, so each load is
        // coalesced) and only then tested
        const bool inr = v < it.y;
        const uint32_t sword = inr ? a.S[v >> 5] : ~0u;
        const uint32_t dg = inr ? a.deg[v] : 0u;
        const int64_t st0 = inr ? a.off[v] : 0;
        const unsigned long long old0 = inr ? a.key[v] : 0ull;
        const bool valid = inr && !((sword >> (v & 31)) & 1u) && dg > 0u;
        if (!ballot(valid)) return;
        const int64_t st = valid ? st0 : 0;
        const unsigned long long old = valid ? old0 : 0ull;
        // unsettled, so its tentative distance is above b; room 0 marks a
        // vertex whose scan has ended
        uint32_t room = valid ? (uint32_t)(old >> 32) - b : 0u;
        smin[l] = ~0ull;
        wave_lds_sync();
        // the run's lists, concatenated, walked kPullWin x 64 edges at a time:
        // every load of those windows is issued before any is used
        const uint32_t d = valid ? dg : 0u;
        const uint32_t inc = wave_incl_sum(d);
        const uint32_t T = __shfl(inc, 63, 64);
        const uint32_t myP = inc - d;  // lanes without edges share the next lane's prefix
        for (uint32_t e0 = 0; e0 < T; e0 += kPullWin * kWave) {
            if (!ballot(room != 0u)) break;  // every scan of the run has ended
            // (edge indices fit in 32 bits)
            uint32_t wk[kPullWin], uk[kPullWin], ok[kPullWin], ek[kPullWin], rk[kPullWin];
#pragma unroll
            for (int k = 0; k < kPullWin; ++k) {
                const uint32_t t = e0 + 64u * k + (uint32_t)l;
                int o = 0;
#pragma unroll
                for (int s2 = 32; s2 >= 1; s2 >>= 1) {
                    const uint32_t pv = __shfl(myP, o + s2, 64);
                    if (pv <= t) o += s2;
                }
                ok[k] = (uint32_t)o;
                ek[k] = __shfl((uint32_t)st, o, 64) + (t - __shfl(myP, o, 64));
                rk[k] = __shfl(room, o, 64);
                wk[k] = (t < T && rk[k] != 0u) ? (uint32_t)a.sw[ek[k]] : 0u;
            }
#pragma unroll
            for (int k = 0; k < kPullWin; ++k) {
                const bool light = wk[k] != 0u && wk[k] <= rk[k];
                uk[k] = light ? a.snbr[ek[k]] : kNone;
                // a heavier edge ends the scan: the rest of the list is heavier
                if (wk[k] > rk[k]) atomicMin(&smin[ok[k]], kScanEnded);
            }
#pragma unroll
            for (int k = 0; k < kPullWin; ++k) {
                if (uk[k] != kNone && test_bit(F, uk[k]))
                    atomicMin(&smin[ok[k]], ((unsigned long long)(b + wk[k]) << 32) | uk[k]);
            }
            wave_lds_sync();
            // a hit ends the scan too: everything after it is a larger key
            if (smin[l] != ~0ull) room = 0u;
        }
        wave_lds_sync();
        const unsigned long long best = smin[l];
        if (valid && best < kScanEnded) {
            if (best < old) {
                a.key[v] = best;  // the run owns v: no other writer this step
                nd = (uint32_t)(best >> 32);
                moved = nd < (uint32_t)(old >> 32);
            }
        }
    } else {
        v = it.x;
        const uint32_t sword = a.S[v >> 5];
        const unsigned long long old0 = a.key[v];
        if ((sword >> (v & 31)) & 1u) return;
        // one piece of a long list, in (weight, neighbour) order; pieces of
        // one list run independently and meet in the atomic minimum
        const uint32_t room = (uint32_t)(old0 >> 32) - b;
        unsigned long long best = ~0ull;
        for (uint32_t e0 = it.z; e0 < it.w; e0 += kPullWin * kWave) {
            uint32_t wk[kPullWin], uk[kPullWin];
#pragma unroll
            for (int k = 0; k < kPullWin; ++k) {
                const uint32_t e = e0 + 64u * k + (uint32_t)l;
                wk[k] = e < it.w ? (uint32_t)a.sw[e] : 0u;
            }
            bool heavy = false;
#pragma unroll
            for (int k = 0; k < kPullWin; ++k) {
                const bool light = wk[k] != 0u && wk[k] <= room;
                heavy |= wk[k] > room;
                uk[k] = light ? a.snbr[e0 + 64u * k + (uint32_t)l] : kNone;
            }
#pragma unroll
            for (int k = 0; k < kPullWin; ++k) {
                if (uk[k] != kNone && test_bit(F, uk[k])) {
                    const unsigned long long c = ((unsigned long long)(b + wk[k]) << 32) | uk[k];
                    best = c < best ? c : best;
                }
            }
#pragma unroll
            for (int s = 32; s >= 1; s >>= 1) {
                const unsigned long long o = shfl64(best, l ^ s);
                best = o < best ? o : best;
            }
            if (best != ~0ull || ballot(heavy)) break;
        }
        if (l == 0 && best != ~0ull && best < a.key[v]) {
            // several pieces of v may race: atomicMin, and a move only on a
            // strictly smaller distance
            const unsigned long long old = atomicMin(&a.key[v], best);
            nd = (uint32_t)(best >> 32);
            moved = nd < (uint32_t)(old >> 32);
        }
    }
    wgb_push(q, moved, v, nd, a);
}

__global__ __launch_bounds__(kRBlock, 8) void wbfs_step_kernel(WbfsArgs a, uint32_t j) {
    __shared__ WgBuckets q;
    __shared__ unsigned long long s_min[kRWaves][kWave];
    __shared__ uint32_t s_b;
    __shared__ unsigned long long s_packed;
    const int l = lane_id();
    const uint32_t bprev = a.ctl[(j + 1) & 1u];
    const uint32_t st = a.ctl[4 + ((j + 1) & 1u)];
    const bool over = a.ctl[3] != 0u;  // a bucket overflowed: the run is void
    const bool pull = (st & kStPull) != 0u && !over;
    if (threadIdx.x < 64) {
        // nextBucket: smallest non-empty slot after the previous bucket (or
        // the previous bucket again when its dense step still has to pull)
        // the found slot's (count, degree sum) comes from the same load;
        // nothing writes slot b while b is current, so it is the value every
        // workgroup sees
        uint32_t b = kDone;
        unsigned long long pk = 0ull;
        if (pull) {
            b = bprev;
            pk = *slot_counter(a, b & (a.NB - 1));
        } else if (bprev != kDone && !over) {
            for (uint32_t k0 = 1; k0 < a.NB; k0 += 64) {
                const uint32_t k = k0 + (uint32_t)l;
                const unsigned long long cv =
                    k < a.NB ? *slot_counter(a, (bprev + k) & (a.NB - 1)) : 0ull;
                const uint64_t mk = ballot((cv >> 32) != 0ull);
                if (mk) {
                    const int fl = first_lane(mk);
                    b = bprev + k0 + (uint32_t)fl;
                    pk = shfl64(cv, fl);
                    break;
                }
            }
        }
        if (l == 0) {
            s_b = b;
            s_packed = pk;
            q.cnt = 0;
        }
    }
    __syncthreads();
    const uint32_t b = s_b;
    const uint32_t slot = b & (a.NB - 1);
    const unsigned long long packed = s_packed;
    const uint32_t cnt = (uint32_t)(packed >> 32);
    const uint32_t E = (uint32_t)packed;
    // every workgroup reads the same (b, cnt, E): a pending pull is decided
    // by the previous launch, and nothing writes slot b while b is current
    bool dense = false;
    if (!pull && b != kDone) {
        if (a.dense_mode == 0u) dense = (unsigned long long)cnt + E > a.dense_thresh;
        else if (a.dense_mode == 2u) dense = true;
        else if (a.dense_mode == 3u) dense = (b & 1u) != 0u;
    }
    const uint32_t npar = (st & kStNextPar) ? 1u : 0u;
    uint32_t mode = kModePush, nst = st & kStNextPar;
    if (pull) {
        mode = kModePull;
        nst = kStClear | ((st & kStPullPar) ? kStClearPar : 0u) | (st & kStNextPar);
    } else if (dense) {
        mode = kModeMark;
        nst = kStPull | (npar ? kStPullPar : 0u) | (npar ? 0u : kStNextPar);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        a.ctl[j & 1u] = b;
        a.ctl[4 + (j & 1u)] = nst;
        if (bprev != kStart && bprev != kDone) *slot_counter(a, bprev & (a.NB - 1)) = 0ull;
        if (b == kDone) {
            a.ctl[2] = 1u;
            if (bprev != kDone) {  // the first launch to find nothing reports it
                host_store(&a.prog[2], over ? 1u : 0u);
                __threadfence_system();
                host_store(&a.prog[1], j + 1);
            }
        } else {
            host_store(&a.prog[0], j + 1);
            if (j < (uint32_t)kWLogCap) {
                host_store(&a.log[4 * j + 0], b);
                host_store(&a.log[4 * j + 1], cnt);
                host_store(&a.log[4 * j + 2], E);
                host_store(&a.log[4 * j + 3], mode);
            }
        }
    }
    const uint32_t gtid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t gstride = gridDim.x * blockDim.x;
    if (st & kStClear) {
        // the pull that read this bitmap ended with the previous launch
        uint32_t* F = a.Fb + ((st & kStClearPar) ? a.fb_stride : 0u);
        for (uint32_t i = gtid; i < a.nw32; i += gstride) F[i] = 0u;
    }
    if (b == kDone) return;
    const int wib = threadIdx.x / kWave;
    if (pull) {
        const uint32_t* F = a.Fb + ((st & kStPullPar) ? a.fb_stride : 0u);
        const uint32_t ntiles = (a.nplan + kRWaves - 1) / kRWaves;
        for (uint32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
            const uint32_t it = tile * kRWaves + (uint32_t)wib;
            if (it < a.nplan) wbfs_pull_item(a, F, b, a.plan[it], s_min[wib], q);
            wgb_maybe_flush(q, a, kRWaves * kWave);
        }
        wgb_flush(q, a);
        return;
    }
    if (cnt > a.C) {
        if (threadIdx.x == 0) a.ctl[3] = 1u;
        return;
    }
    const uint32_t* Q = a.Qs + (size_t)slot * a.C;
    if (dense) {
        // mark bucket b's live vertices (they are settled now) for the pull
        uint32_t* F = a.Fb + (npar ? a.fb_stride : 0u);
        for (uint32_t i = gtid; i < cnt; i += gstride) {
            const uint32_t u = Q[i];
            if ((uint32_t)(a.key[u] >> 32) == b) {
                atomicOr(&F[u >> 5], 1u << (u & 31));
                atomicOr(&a.S[u >> 5], 1u << (u & 31));
            }
        }
        return;
    }
    const uint32_t* P = a.Ps + (size_t)slot * a.C;
    const uint32_t nwaves = gridDim.x * kRWaves;
    RelaxPolicy pol{&a, &q, b};
    const uint32_t cap = min(a.chunk_cap, (uint32_t)(kWgCapW / (2 * kRWaves)));
    const uint32_t wc = wave_chunk(E, nwaves, cap);
    const uint32_t nchunks = (E + wc - 1) / wc;
    const uint32_t ntiles = (nchunks + kRWaves - 1) / kRWaves;
    // workgroup-uniform tiles of 16 chunks, so the LDS buffer can be flushed
    // between tiles
    for (uint32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const uint32_t c = tile * kRWaves + wib;
        if (c < nchunks) {
            const uint32_t eb = c * wc;
            expand_range(Q, P, cnt, E, a.off, eb, min(E, eb + wc), pol);
        }
        wgb_maybe_flush(q, a, kRWaves * wc);
    }
    wgb_flush(q, a);
}

__global__ __launch_bounds__(kBlock) void wbfs_finalize_kernel(const unsigned long long* key,
                                                               int64_t n, uint32_t* dist,
                                                               int32_t* parent) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = tid; v < n; v += stride) {
        const unsigned long long k = key[v];
        dist[v] = (uint32_t)(k >> 32);
        parent[v] = (int32_t)(uint32_t)k;
    }
}

// One weighted BFS on workspace w.  Sets *overflow (and leaves the outputs
// unspecified) when a bucket outgrew the workspace's capacity.
int run_wbfs_ws(gbgpu_graph g, WbfsWs* w, int32_t src, uint32_t* dist, int32_t* parent,
                const gbgpu_opts& o, gbgpu_stats* st, hipStream_t stream, bool* overflow) {
    const double t0 = now_ms();
    GB_TRY(ensure_wsort(g, stream));
    WbfsArgs a;
    a.off = g->off;
    a.nbr = g->nbr;
    a.wt = g->w;
    a.snbr = g->wsort_nbr;
    a.sw = g->wsort_w;
    a.deg = g->deg;
    a.key = w->key;
    a.Qs = w->Qs;
    a.Ps = w->Ps;
    a.sc = w->sc;
    a.S = w->S;
    a.Fb = w->Fb;
    a.ctl = w->ctl;
    a.prog = w->hl.d;
    a.log = w->hl.d + kHostLogOff;
    a.plan = g->plan;
    a.n = g->n;
    a.NB = w->NB;
    a.C = w->C;
    a.chunk_cap = (uint32_t)o.wave_chunk;
    a.nw32 = (uint32_t)((g->n + 31) / 32);
    a.fb_stride = (uint32_t)(wal((size_t)((g->n + 63) / 64) * 8) / 4);
    a.nplan = g->nplan;
    a.dense_mode = (uint32_t)(o.force_direction == 1 ? 1 : o.force_direction == 2 ? 2
                              : o.force_direction == 3 ? 3 : 0);
    // a bucket goes dense when its entries + their degrees exceed m / tau;
    // unless the caller sets tau, 10 (RMAT scale 24, w < 24: 7.3 ms per
    // source against 8.2 at 20 and 7.9 at 5; the dense steps cannot stop
    // at the first frontier neighbour the way BFS's do, so they pay off
    // only for heavier buckets)
    const int tau = o.reserved[kTauDefaulted] ? kWbfsTau : std::max(o.tau, 1);
    a.dense_thresh = (unsigned long long)g->m / (unsigned long long)tau;
    const int igrid = (int)std::min<int64_t>(std::max<int64_t>((g->n + kBlock - 1) / kBlock, 64), 4096);
    hipLaunchKernelGGL(wbfs_init_kernel, dim3(igrid), dim3(kBlock), 0, stream, a, (uint32_t)src);
    GB_HIP(hipGetLastError());
    const int64_t work = std::max<int64_t>(1, g->m / 4096);
    const int grid = (int)std::min<int64_t>(work, o.grid);
    *overflow = false;
    volatile uint32_t* hp = w->hl.h;
    hp[0] = 0;
    hp[1] = 0;
    hp[2] = 0;
    if (o.profile) GB_HIP(hipEventRecord(w->ev0, stream));
    // at most one bucket per distinct distance, two launches per dense bucket
    const int64_t max_launches = 2 * g->n + 4;
    int64_t launches = 0;
    GB_TRY(run_pipeline(
        hp, stream, o.rounds_per_sync, max_launches,
        [&](int64_t jj) {
            hipLaunchKernelGGL(wbfs_step_kernel, dim3(grid), dim3(kRBlock), 0, stream, a,
                               (uint32_t)jj);
        },
        &launches));
    if (o.profile) GB_HIP(hipEventRecord(w->ev1, stream));
    // (after an overflow the outputs are rewritten by the rerun)
    hipLaunchKernelGGL(wbfs_finalize_kernel, dim3(igrid), dim3(kBlock), 0, stream, w->key, g->n,
                       dist, parent);
    GB_HIP(hipGetLastError());
    GB_HIP(hipStreamSynchronize(stream));
    const uint32_t steps = hp[1] - 1;
    w->last_steps = steps;
    if (hp[2]) {
        *overflow = true;
        return GBGPU_OK;
    }
    if (st) {
        memset(st, 0, sizeof(*st));
        if (o.profile) {
            float ms = 0.f;
            GB_HIP(hipEventElapsedTime(&ms, w->ev0, w->ev1));
            st->kernel_ms = ms;
        }
        const uint32_t* lg = w->hl.h + kHostLogOff;
        uint32_t peak = 0;
        for (uint32_t i = 0; i < std::min<uint32_t>(steps, (uint32_t)kWLogCap); ++i) {
            if (lg[4 * i + 3] == kModePull) {
                st->pull_rounds++;
                continue;
            }
            st->rounds++;
            if (lg[4 * i + 3] == kModePush) st->push_rounds++;
            st->edges_examined += lg[4 * i + 2];
            peak = std::max(peak, lg[4 * i + 1]);
        }
        // the fill of every bucket is known only when every step was logged
        st->bucket_peak = steps <= (uint32_t)kWLogCap ? (int32_t)peak : 0;
        st->launches = (int32_t)launches;
        st->wall_ms = now_ms() - t0;
    }
    return GBGPU_OK;
}

int run_wbfs(gbgpu_graph g, int32_t src, uint32_t* dist, int32_t* parent, const gbgpu_opts& o,
             gbgpu_stats* st, hipStream_t stream) {
    const double t0 = now_ms();
    const uint32_t NB = wbfs_window(g->maxw, o.bucket_window);
    uint32_t C = o.bucket_capacity > 0 ? (uint32_t)std::min<int64_t>(o.bucket_capacity, g->n)
                                       : wbfs_default_capacity(g->n);
    if (g->wbfs && g->wbfs->NB == NB && g->wbfs->C >= C && o.bucket_capacity <= 0) C = g->wbfs->C;
    int retries = 0;
    for (;;) {
        GB_TRY(ensure_wbfs_ws(g, NB, C));
        bool overflow = false;
        GB_TRY(run_wbfs_ws(g, g->wbfs, src, dist, parent, o, st, stream, &overflow));
        if (!overflow) break;
        if (C >= (uint32_t)g->n)
            return set_error(GBGPU_E_HIP, "bucket overflow at full capacity (internal error)");
        C = (uint32_t)std::min<int64_t>(g->n, (int64_t)C * 2);
        ++retries;
    }
    if (st) {
        st->retries = retries;
        st->wall_ms = now_ms() - t0;
    }
    return GBGPU_OK;
}

int wbfs_step_log(gbgpu_graph g, uint32_t* out, int32_t max_steps, int32_t* nsteps) {
    if (!g->wbfs) { *nsteps = 0; return GBGPU_OK; }
    const int32_t r = (int32_t)std::min<int64_t>(
        std::min<int64_t>(max_steps, kWLogCap), g->wbfs->last_steps);
    memcpy(out, g->wbfs->hl.h + kHostLogOff, (size_t)r * 16);
    *nsteps = r;
    return GBGPU_OK;
}

}  // namespace gb
