// Batched BFS: many sources, possibly on many graphs, in one launch per round.
//
// The paper's strongly-connected-components algorithm runs the searches
// from all active centers simultaneously, one edgeMap per round, each
// search adding in every round exactly the labels it would add alone, and
// keeps the first phase's reachability in bit-vectors; here the labels are
// the bits of a per-vertex mask, one bit per source.
//
// Sources are packed 64 to a group; a group is (graph, up to 64 sources) and
// every vertex of the group's graph carries three 64-bit masks: visited VM,
// frontier F_r and next frontier F_{r+1} (bit j = source j).  One launch per
// round processes every active group of every graph: the work of all groups
// is laid out in one index space and each wavefront takes units from it.
// Each group chooses its own direction on the device from its frontier
// totals, exactly like the single-source edgeMap switch:
//   push (sparse): the frontier list (ids + degree prefix) is expanded edge by
//     edge; for an edge (u, v), the bits of F_r[u] that v has not seen are
//     OR-ed into F_{r+1}[v] and every such bit j takes the atomic minimum of
//     its pair entry with (r + 1, u);
//   pull (dense): every vertex with unseen bits scans its ascending list; the
//     first neighbour u that carries bit j in F_r becomes parent_j[v] (a
//     wavefront prefix-OR finds first contributors when a whole wavefront
//     scans one list), with early exit once every unseen bit is found.
// Both rules give parent_j[v] = min{u in N(v) : D_j[u] = D_j[v] - 1}, so each
// row equals the single-source BFS from source j.  A pair (v, j) is written
// once, in the round r that finds it, as one entry (arrival round r + 1,
// parent; 4 or 8 bytes, see MsGroupDev::E): D_j[v] = r + 1, the round whose
// frontier holds bit j of v.
// Groups finish independently; a finished group costs nothing.

#include "common.h"
#include "emit.h"
#include "gridbar.h"

namespace gb {

constexpr int kMaxGroups = 64;
// last round a group with 4-byte pair entries may run (its arrivals, at most
// this round + 1, fill the 8-bit round field)
constexpr uint32_t kNarrowRounds = 254;
// 64-edge windows a wavefront of the dense scan loads before it updates: 2,
// or 6 on graphs of average degree at most 8, where a 64-vertex run's edges
// then come in one step (256^3 torus, 64 sources: 375 against 408 ms; on
// RMAT-24 six windows cost 19.5 against 18.9 ms, the early exits coming a
// step later)
constexpr int kMsWin = 2;
constexpr int kMsWinSparse = 6;

struct MsGroupDev {
    const int64_t* off;
    const int32_t* nbr;
    const uint32_t* deg;
    int64_t n;
    uint64_t dense_thresh;
    uint64_t m;                 // stored edges
    unsigned long long kmask;   // bits of the sources in this group (kused of them)
    unsigned long long* VM;     // n
    unsigned long long* F[3];   // n each
    uint32_t* Q[2];             // n + 64 each
    uint32_t* P[2];
    unsigned long long* ctl;    // [0..3] qcnt, [4..7] qover, then 4 x kSpread x kSpreadStride totals
    int32_t* const* drow;       // 64 row pointers (dist), device array
    int32_t* const* prow;       // 64 row pointers (parent), device array
    const uint4* plan;          // dense-scan work items of the graph
    uint32_t nplan;
    uint32_t k;                 // capacity: sources the staging holds per vertex
    uint32_t kused;             // sources in the group so far (bits 0 .. kused-1)
    // vertex-major pair entries E[v * k + j], written when the pair is found
    // and ~0 until then: (round of arrival << 32) | parent in 8 bytes, or,
    // when narrow, (round << 24) | parent in 4 bytes (graphs of at most 2^24
    // vertices, groups that take no arrivals, rounds up to kNarrowRounds)
    void* E;
    uint32_t narrow;
    uint32_t* start;            // round at which source j joined the group (64)
};

__device__ __host__ __forceinline__ unsigned long long* ent64(const MsGroupDev& G) {
    return (unsigned long long*)G.E;
}
__device__ __host__ __forceinline__ uint32_t* ent32(const MsGroupDev& G) { return (uint32_t*)G.E; }

struct MsArgs {
    MsGroupDev* groups;
    unsigned long long* ovf;  // bit gi: narrow group gi reached round kNarrowRounds + 1
    int32_t ngroups;
    int32_t force_dir;
    int32_t light;
    uint32_t chunk_cap;
    uint32_t* log;   // per (round, group): direction
};

struct MultiWs {
    void* block = nullptr;
    size_t bytes = 0;
    void* host_pin = nullptr;
};

void free_multi_ws(MultiWs* w) {
    if (!w) return;
    if (w->block) (void)hipFree(w->block);
    if (w->host_pin) (void)hipHostFree(w->host_pin);
    delete w;
}

__device__ __forceinline__ unsigned long long* ms_tot(const MsGroupDev& G, uint32_t slot) {
    return G.ctl + 8 + (size_t)(slot & 3u) * kSpread * kSpreadStride;
}

// 64-bit exclusive prefix OR across the wavefront (lane order).
__device__ __forceinline__ unsigned long long wave_excl_or64(unsigned long long x) {
    const int l = lane_id();
    unsigned long long inc = x;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        unsigned long long y = shfl64(inc, max(l - d, 0));
        if (l >= d) inc |= y;
    }
    unsigned long long ex = shfl64(inc, max(l - 1, 0));
    return l == 0 ? 0ull : ex;
}

__global__ __launch_bounds__(kBlock) void ms_init_kernel(MsGroupDev* groups, int32_t gi,
                                                        const uint32_t* srcs, int32_t k) {
    const MsGroupDev G = groups[gi];
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = tid; v < G.n; v += stride) {
        G.VM[v] = 0ull;
        G.F[0][v] = 0ull;
        G.F[1][v] = 0ull;
        G.F[2][v] = 0ull;
    }
    // pair entries start at ~0 so that sparse rounds can take atomicMin (the
    // final transpose reads only reached pairs)
    const int64_t words = G.n * (int64_t)G.k * (G.narrow ? 1 : 2);  // 4-byte words
    uint4* e4 = (uint4*)G.E;
    for (int64_t i = tid; i < words / 4; i += stride) e4[i] = make_uint4(~0u, ~0u, ~0u, ~0u);
    for (int64_t i = (words / 4) * 4 + tid; i < words; i += stride) ((uint32_t*)G.E)[i] = ~0u;
    for (int64_t i = tid; i < 8 + 4 * kSpread * kSpreadStride; i += stride) G.ctl[i] = 0ull;
}

// After init: frontier F_0 = source bits, list Q_0 = distinct sources; the
// sources' own entries (distance 0, parent itself, visited) are set here so
// that an isolated source needs no traversal work.
__global__ void ms_seed_kernel(MsGroupDev* groups, int32_t gi, const uint32_t* srcs, int32_t k,
                               unsigned long long* ovf) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const MsGroupDev G = groups[gi];
    if (ovf) *ovf = 0ull;
    uint32_t cnt = 0, edges = 0;
    for (int j = 0; j < k; ++j) {
        const uint32_t s = srcs[j];
        if (G.F[0][s] == 0ull) {
            G.Q[0][cnt] = s;
            G.P[0][cnt] = edges;
            ++cnt;
            edges += G.deg[s];
        }
        G.F[0][s] |= 1ull << j;
        G.VM[s] |= 1ull << j;
        // round 0, parent itself
        if (G.narrow) ent32(G)[(size_t)s * G.k + j] = s;
        else ent64(G)[(size_t)s * G.k + j] = s;
    }
    for (int j = 0; j < 64; ++j) G.start[j] = 0;
    G.ctl[0] = ((unsigned long long)cnt << 32) | edges;  // qcnt slot 0
    ms_tot(G, 0)[0] = ((unsigned long long)cnt << 32) | edges;
}

// Before sources join a group whose frontier ran empty: the rounds since
// then skipped their frontier bookkeeping, so one of the three frontier
// arrays may still hold the last non-empty frontier.
__global__ __launch_bounds__(kBlock) void ms_clear_frontiers_kernel(MsGroupDev* groups, int32_t gi) {
    const MsGroupDev G = groups[gi];
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = tid; v < G.n; v += stride) {
        G.F[0][v] = 0ull;
        G.F[1][v] = 0ull;
        G.F[2][v] = 0ull;
    }
}

// Round-boundary admission: sources j0 .. j0+cnt-1 join a running group
// before round r (the stream is idle between rounds r-1 and r).  Each new
// source enters round r's frontier (and its list, when the group keeps
// one) exactly as a source enters round 0, and its rounds are counted from
// r: row j's distance is the round of arrival minus start[j].  A group
// whose frontier was empty gets a fresh (valid) list.
__global__ void ms_join_kernel(MsGroupDev* groups, int32_t gi, uint32_t r, const uint32_t* srcs,
                               uint32_t j0, uint32_t cnt) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    MsGroupDev& G = groups[gi];
    unsigned long long* F = G.F[r % 3];
    unsigned long long* tot = ms_tot(G, r);
    unsigned long long t = 0;
    for (int c = 0; c < kSpread; ++c) t += tot[(size_t)c * kSpreadStride];
    if ((t >> 32) == 0) G.ctl[4 + (r & 3u)] = 0ull;
    const bool qvalid = G.ctl[4 + (r & 3u)] == 0ull;
    uint32_t qn = (uint32_t)(t >> 32), edges = (uint32_t)t;
    unsigned long long add = 0, bits = 0;
    for (uint32_t i = 0; i < cnt; ++i) {
        const uint32_t s = srcs[i];
        const uint32_t j = j0 + i;
        if (F[s] == 0ull) {
            if (qvalid) {
                G.Q[r & 1u][qn] = s;
                G.P[r & 1u][qn] = edges;
            }
            ++qn;
            edges += G.deg[s];
            add += (1ull << 32) | G.deg[s];
        }
        F[s] |= 1ull << j;
        G.VM[s] |= 1ull << j;
        ent64(G)[(size_t)s * G.k + j] = ((unsigned long long)r << 32) | s;  // never narrow
        G.start[j] = r;
        bits |= 1ull << j;
    }
    tot[0] += add;
    if (qvalid) G.ctl[r & 3u] += add;
    G.kmask |= bits;
    G.kused = j0 + cnt;
}

// vertex rows of a transpose tile each thread loads
constexpr int kTileRows = 64 / (kBlock / 64);

// Thread t's share of a 64-vertex tile of pair entries (column t % 64, rows
// t / 64 + 16 i): parent and round of arrival of each reached pair.  Every
// load is issued before any is used, so a thread keeps kTileRows reads in
// flight; pairs the search never reached are not read (their row entries
// are written as unreachable).
template <class T>
__device__ __forceinline__ void ms_load_tile(const T* E, int64_t v0, int nv, int k, int ku, int t,
                                             const unsigned long long* tv, uint32_t* lp,
                                             uint32_t* ld) {
    const int j = t & 63;
    T e[kTileRows];
#pragma unroll
    for (int i = 0; i < kTileRows; ++i) {
        const int vi = (t >> 6) + i * (kBlock / 64);
        const bool ok = vi < nv && j < ku && ((tv[vi < nv ? vi : 0] >> j) & 1ull);
        e[i] = ok ? E[(size_t)(v0 + vi) * k + j] : (T)0;
    }
#pragma unroll
    for (int i = 0; i < kTileRows; ++i) {
        if constexpr (sizeof(T) == 4) {
            lp[i] = (uint32_t)e[i] & 0xFFFFFFu;
            ld[i] = (uint32_t)e[i] >> 24;
        } else {
            lp[i] = (uint32_t)e[i];
            ld[i] = (uint32_t)(e[i] >> 32);
        }
    }
}

// Final layout: row j of the caller's output = source j.  Each workgroup
// moves a tile of 64 vertices x kused sources through LDS so both the
// vertex-major reads and the row writes are coalesced; unreached pairs get
// (INT32_MAX, -1); a distance is the round of arrival minus the round the
// source joined (0 unless it joined a running group).
__global__ __launch_bounds__(kBlock) void ms_transpose_kernel(MsGroupDev* groups, int32_t gi) {
    __shared__ uint32_t tp[64][65];
    __shared__ uint32_t td[64][65];
    __shared__ unsigned long long tv[64];
    __shared__ int32_t* rd[64];
    __shared__ int32_t* rp[64];
    __shared__ uint32_t st[64];
    const MsGroupDev G = groups[gi];
    const int k = (int)G.k;       // staging stride
    const int ku = (int)G.kused;  // rows to write
    const int t = threadIdx.x;
    if (t < ku) {
        rd[t] = G.drow[t];
        rp[t] = G.prow[t];
        st[t] = G.start[t];
    }
    // thread t handles source column (t % 64) in the load phase and writes
    // four consecutive vertices of row (t / 16 + 16 * pass) in the store phase
    for (int64_t v0 = (int64_t)blockIdx.x * 64; v0 < G.n; v0 += (int64_t)gridDim.x * 64) {
        const int nv = (int)min<int64_t>(64, G.n - v0);
        __syncthreads();
        if (t < nv) tv[t] = G.VM[v0 + t];
        __syncthreads();
        const int j = t & 63;
        uint32_t lp[kTileRows], ld[kTileRows];
        if (G.narrow)
            ms_load_tile(ent32(G), v0, nv, k, ku, t, tv, lp, ld);
        else
            ms_load_tile(ent64(G), v0, nv, k, ku, t, tv, lp, ld);
#pragma unroll
        for (int i = 0; i < kTileRows; ++i) {
            const int vi = (t >> 6) + i * (kBlock / 64);
            tp[vi][j] = lp[i];
            td[vi][j] = ld[i];
        }
        __syncthreads();
        const int q = t & 15;  // four vertices 4q .. 4q+3
        for (int row = t >> 4; row < ku; row += kBlock / 16) {
            const int vb = 4 * q;
            if (vb >= nv) continue;
            int32_t dv[4], pv[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int vi = vb + i;
                const bool reached = vi < nv && ((tv[vi < nv ? vi : 0] >> row) & 1ull);
                dv[i] = reached ? (int32_t)(td[vi][row] - st[row]) : INT32_MAX;
                pv[i] = reached ? (int32_t)tp[vi][row] : -1;
            }
            int32_t* drow = rd[row] + v0 + vb;
            int32_t* prow = rp[row] + v0 + vb;
            if (vb + 4 <= nv && (((uintptr_t)drow | (uintptr_t)prow) & 15) == 0) {
                *(int4*)drow = make_int4(dv[0], dv[1], dv[2], dv[3]);
                *(int4*)prow = make_int4(pv[0], pv[1], pv[2], pv[3]);
            } else {
                for (int i = 0; i < 4 && vb + i < nv; ++i) {
                    drow[i] = dv[i];
                    prow[i] = pv[i];
                }
            }
        }
    }
}

constexpr uint32_t kMsEmit = 256;  // next-list entries a wavefront buffers

struct MsEmitBuf {
    uint32_t v[kMsEmit];
    uint32_t d[kMsEmit];
};

// A wavefront's buffer of next-list entries for one group: the dense scan
// appends the vertices it finds in LDS and reserves their room in the
// group's list with one atomic per flush.  The list's counter is a single
// address for the whole grid, so one reservation per plan item serialised
// (a round whose frontier shrinks to ~10^5 scattered vertices spent about a
// millisecond on them).
struct MsEmitter {
    MsEmitBuf* b;
    uint32_t n;  // buffered entries (wave-uniform)
};

// Writes the buffered entries (ids, degree prefix) to `out` after one
// reservation; nothing is written once the list has been abandoned.
// Wave-uniform.
__device__ __forceinline__ void ms_emit_flush(MsEmitter& e, const QueueOut& out) {
    if (e.n == 0u) return;
    wave_lds_sync();
    const int l = lane_id();
    const uint32_t n = e.n;
    uint32_t ds = 0;
    for (uint32_t i0 = 0; i0 < n; i0 += 64u) {
        const uint32_t i = i0 + (uint32_t)l;
        ds += wave_sum(i < n ? e.b->d[i] : 0u);
    }
    unsigned long long packed = ~0ull;
    if (l == 0 && *(volatile unsigned long long*)out.qover == 0) {
        packed = atomicAdd(out.qcnt, ((unsigned long long)n << 32) | ds);
        if ((uint64_t)(packed >> 32) + n + (uint32_t)packed + ds > out.qlimit) {
            *out.qover = 1ull;
            packed = ~0ull;
        }
    }
    packed = shfl64(packed, 0);
    if (packed != ~0ull) {
        const uint32_t pos = (uint32_t)(packed >> 32);
        uint32_t dp = (uint32_t)packed;
        for (uint32_t i0 = 0; i0 < n; i0 += 64u) {
            const uint32_t i = i0 + (uint32_t)l;
            const uint32_t x = i < n ? e.b->d[i] : 0u;
            const uint32_t inc = wave_incl_sum(x);
            if (i < n) {
                out.Q[pos + i] = e.b->v[i];
                out.P[pos + i] = dp + inc - x;
            }
            dp += __shfl(inc, 63, 64);
        }
    }
    wave_lds_sync();  // every lane has read the buffer before it refills
    e.n = 0u;
}

// Appends the lanes of m (those with take set) with their degrees; `out` is
// the list the buffer holds entries for.
__device__ __forceinline__ void ms_emit_add(MsEmitter& e, const QueueOut& out, bool take,
                                            uint32_t v, uint32_t dv, uint64_t m) {
    const uint32_t k = (uint32_t)__popcll(m);
    if (e.n + k > kMsEmit) ms_emit_flush(e, out);
    if (take) {
        const uint32_t p = e.n + mbcnt(m);
        e.b->v[p] = v;
        e.b->d[p] = dv;
    }
    e.n += k;
}

struct MsPushPolicy {
    const MsGroupDev* G;
    const unsigned long long* Fc;
    unsigned long long* Fn;
    const QueueOut* out;
    MsEmitter* em;
    uint32_t arrive;  // round in which the pairs found now enter the frontier
    uint32_t found;
    uint32_t dsum;
    static constexpr bool kSkipDead = false;

    __device__ __forceinline__ uint32_t aux(uint32_t) const { return 1u; }

    __device__ __forceinline__ void edge(bool act, uint32_t u, uint32_t, int64_t e, bool) {
        bool claim = false;
        uint32_t v = 0, dv = 0;
        if (act) {
            v = (uint32_t)G->nbr[e];
            const unsigned long long seen = G->VM[v] | Fc[v];
            const unsigned long long cand = Fc[u] & G->kmask & ~seen;
            if (cand) {
                const unsigned long long old = atomicOr(&Fn[v], cand);
                claim = old == 0ull;
                // every pair found this round arrives in round r + 1: the
                // minimum entry holds the smallest parent
                unsigned long long bits = cand;
                while (bits) {
                    const int j = __ffsll((long long)bits) - 1;
                    bits &= bits - 1;
                    const size_t at = (size_t)v * G->k + j;
                    if (G->narrow) {
                        const uint32_t key = (arrive << 24) | u;
                        uint32_t* pp = ent32(*G) + at;
                        if (key < *pp) atomicMin(pp, key);
                    } else {
                        const unsigned long long key = ((unsigned long long)arrive << 32) | u;
                        unsigned long long* pp = ent64(*G) + at;
                        if (key < *pp) atomicMin(pp, key);
                    }
                }
                if (claim) dv = G->deg[v];
            }
        }
        const uint64_t m = ballot(claim);
        if (m) {
            ms_emit_add(*em, *out, claim, v, dv, m);
            if (claim) {
                found += 1;
                dsum += dv;
            }
        }
    }
    __device__ __forceinline__ void window_done() {}
};

__device__ __forceinline__ unsigned long long shfl_up64(unsigned long long x, int d) {
    const uint32_t lo = __shfl_up((uint32_t)x, d, 64);
    const uint32_t hi = __shfl_up((uint32_t)(x >> 32), d, 64);
    return ((unsigned long long)hi << 32) | lo;
}

__device__ __forceinline__ unsigned long long wave_or64(unsigned long long x) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        const uint32_t lo = __shfl_xor((uint32_t)x, d, 64);
        const uint32_t hi = __shfl_xor((uint32_t)(x >> 32), d, 64);
        x |= ((unsigned long long)hi << 32) | lo;
    }
    return x;
}

// row_l[j] = val_l for every lane l and every set bit j of bits_l
// (wave-uniform call).  The stores are dealt out over the lanes in slot
// order, lane l's bits taking consecutive slots, so one store instruction
// writes up to 64 entries and the entries of one row sit in neighbouring
// lanes: a row costs a few cache-line writes instead of one write request
// per bit (a loop over each lane's own bits issues one store per bit with
// every lane on a different row).
template <class T>
__device__ __forceinline__ void wave_store_bits(unsigned long long bits, T* row, T val) {
    const int l = lane_id();
    const uint32_t c = (uint32_t)__popcll(bits);
    const uint32_t inc = wave_incl_sum(c);
    const uint32_t total = __shfl(inc, 63, 64);
    const uint32_t ex = inc - c;
    for (uint32_t s0 = 0; s0 < total; s0 += 64u) {
        const uint32_t s = s0 + (uint32_t)l;
        // slot s belongs to the last lane whose first slot is <= s; that
        // lane has at least s - ex + 1 bits, since the next lane starts
        // after s
        int o = 0;
#pragma unroll
        for (int st = 32; st >= 1; st >>= 1)
            if (__shfl(ex, o + st, 64) <= s) o += st;
        const unsigned long long b = shfl64(bits, o);
        const uint64_t rp = shfl64((uint64_t)(uintptr_t)row, o);
        T v;
        if constexpr (sizeof(T) == 8) v = (T)shfl64((uint64_t)val, o);
        else v = (T)__shfl((uint32_t)val, o, 64);
        const uint32_t k = s - __shfl(ex, o, 64);
        if (s < total) {
            const uint32_t lo = (uint32_t)__popc((uint32_t)b);
            const uint32_t j = k < lo ? select_bit((uint32_t)b, k)
                                      : 32u + select_bit((uint32_t)(b >> 32), k - lo);
            ((T*)(uintptr_t)rp)[j] = v;
        }
    }
}


// Dense scan of one plan item that is a run of <= 64 vertices: the run's
// edges are contiguous, so the wavefront walks them 64 at a time (coalesced
// neighbour loads) and finds, for every vertex and every unseen bit, the
// first neighbour in ascending order that carries the bit: a segmented
// prefix-OR over the lanes of each vertex gives first contributors within a
// window, and a per-vertex accumulator carries earlier windows.  A vertex
// stops being scanned once all its unseen bits are found.
template <int W>
__device__ __forceinline__ void ms_pull_run(const MsGroupDev& G, uint32_t r, uint4 it,
                                            const unsigned long long* __restrict__ Fc,
                                            unsigned long long* Fn, MsEmitter& em,
                                            const QueueOut& out, bool emit, uint32_t& found,
                                            uint32_t& dsum) {
    const int l = lane_id();
    const uint32_t vb = it.x, nv = it.y - it.x;
    const bool in = (uint32_t)l < nv;
    const uint32_t v = vb + (uint32_t)l;
    const int64_t base = G.off[vb];
    const uint32_t T = (uint32_t)(G.off[it.y] - base);
    int64_t o0 = 0, o1 = 0;
    unsigned long long f = 0, vm = 0;
    if (in) {
        o0 = G.off[v];
        o1 = G.off[v + 1];
        f = Fc[v];
        vm = G.VM[v];
    }
    const uint32_t s = in ? (uint32_t)(o0 - base) : 0xFFFFFFFFu;
    const uint32_t d = (uint32_t)(o1 - o0);
    if (in && f) G.VM[v] = vm | f;  // fold of F_r
    const unsigned long long need = (in && d) ? (G.kmask & ~(vm | f)) : 0ull;
    unsigned long long acc = 0ull;
    uint64_t live = ballot(need != 0ull);
    auto owner = [&](uint32_t x) {
        int o = 0;
#pragma unroll
        for (int st = 32; st >= 1; st >>= 1) {
            const uint32_t pv = __shfl(s, o + st, 64);
            if (pv <= x) o += st;
        }
        return o;
    };
    uint32_t e = 0;
    while (e < T && live) {
        const int oe = owner(e);
        if (!((live >> oe) & 1ull)) {
            const uint64_t after = oe == 63 ? 0ull : (live & (~0ull << (oe + 1)));
            if (!after) break;
            e = max(e, __shfl(s, first_lane(after), 64));
            continue;
        }
        // W windows: owners, then all loads, then the ordered updates
        int ow[W];
        uint32_t u[W];
        unsigned long long fu[W];
#pragma unroll
        for (int k = 0; k < W; ++k) {
            const uint32_t t = e + 64u * k + (uint32_t)l;
            ow[k] = owner(t);
            const bool act = t < T && ((live >> ow[k]) & 1ull);
            u[k] = act ? (uint32_t)G.nbr[base + t] : kNone;
        }
#pragma unroll
        for (int k = 0; k < W; ++k) fu[k] = u[k] != kNone ? Fc[u[k]] : 0ull;
#pragma unroll
        for (int k = 0; k < W; ++k) {
            const uint32_t eb = e + 64u * k;
            if (eb >= T) break;
            const int o = ow[k];
            const unsigned long long acc_o = shfl64(acc, o);
            const unsigned long long need_o = shfl64(need, o);
            const unsigned long long add = fu[k] & need_o & ~acc_o;
            const uint32_t so = __shfl(s, o, 64);
            const int seg = so > eb ? (int)(so - eb) : 0;
            unsigned long long incl = add;
#pragma unroll
            for (int st = 1; st < 64; st <<= 1) {
                const unsigned long long y = shfl_up64(incl, st);
                if (l - st >= seg) incl |= y;
            }
            unsigned long long excl = shfl_up64(incl, 1);
            if (l - 1 < seg) excl = 0ull;
            const size_t row = (size_t)(vb + (uint32_t)o) * G.k;
            if (G.narrow)
                wave_store_bits(add & ~excl, ent32(G) + row, ((r + 1u) << 24) | u[k]);
            else
                wave_store_bits(add & ~excl, ent64(G) + row,
                                ((unsigned long long)(r + 1u) << 32) | u[k]);
            // each vertex takes the OR of its lanes in this window
            uint32_t last = 0;
            bool hasw = false;
            if (in && d) {
                const uint32_t a = s > eb ? s - eb : 0u;
                const uint32_t endl = min(s + d, T);
                if (s < eb + 64u && endl > eb) {
                    last = min(endl - eb, 64u) - 1u;
                    hasw = a <= last;
                }
            }
            const unsigned long long tot = shfl64(incl, (int)last);
            if (hasw) acc |= tot;
        }
        live = ballot(need != 0ull && acc != need);
        e += 64u * W;
    }
    const bool got = acc != 0ull;
    if (in && got) {
        Fn[v] = acc;
        found += 1;
        dsum += d;
    }
    const uint64_t m = ballot(got);
    if (m && emit) ms_emit_add(em, out, got, v, d, m);
}

// Dense scan of a piece of one long list: first contributors within the
// piece, then atomicMin per bit across pieces (pieces of one list may run
// concurrently); the next-frontier bits are OR-ed atomically and the piece
// that sets the first bit counts the vertex.
__device__ __forceinline__ void ms_pull_piece(const MsGroupDev& G, uint32_t r, uint4 it,
                                              const unsigned long long* __restrict__ Fc,
                                              unsigned long long* Fn, MsEmitter& em,
                                              const QueueOut& out, bool emit, uint32_t& found,
                                              uint32_t& dsum) {
    const int l = lane_id();
    const uint32_t v = it.x;
    const int64_t ob = G.off[v], oe = G.off[v + 1];
    const unsigned long long f = Fc[v], vm = G.VM[v];
    if ((int64_t)it.z == ob && f && l == 0) G.VM[v] = vm | f;  // the first piece folds v
    const unsigned long long need = G.kmask & ~(vm | f);
    unsigned long long acc = 0ull;
    for (uint32_t e = it.z; e < it.w && need && acc != need; e += 128u) {
        const uint32_t t0 = e + (uint32_t)l, t1 = e + 64u + (uint32_t)l;
        const uint32_t u0 = t0 < it.w ? (uint32_t)G.nbr[t0] : kNone;
        const uint32_t u1 = t1 < it.w ? (uint32_t)G.nbr[t1] : kNone;
        const unsigned long long f0 = u0 != kNone ? Fc[u0] : 0ull;
        const unsigned long long f1 = u1 != kNone ? Fc[u1] : 0ull;
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const uint32_t u = k ? u1 : u0;
            const unsigned long long add = (k ? f1 : f0) & need & ~acc;
            unsigned long long first = add & ~wave_excl_or64(add);
            // pieces of one list may run concurrently: atomic minimum of the
            // pair entry (every candidate this round has the same arrival)
            while (first) {
                const int j = __ffsll((long long)first) - 1;
                first &= first - 1;
                const size_t at = (size_t)v * G.k + j;
                if (G.narrow) {
                    const uint32_t key = ((r + 1u) << 24) | u;
                    uint32_t* pp = ent32(G) + at;
                    if (key < *pp) atomicMin(pp, key);
                } else {
                    const unsigned long long key = ((unsigned long long)(r + 1u) << 32) | u;
                    unsigned long long* pp = ent64(G) + at;
                    if (key < *pp) atomicMin(pp, key);
                }
            }
            acc |= wave_or64(add);
        }
    }
    bool claim = false;
    if (l == 0 && acc) claim = atomicOr(&Fn[v], acc) == 0ull;
    claim = __shfl((int)claim, 0, 64) != 0;
    if (claim && l == 0) {
        found += 1;
        dsum += (uint32_t)(oe - ob);
    }
    const uint64_t m = ballot(claim && l == 0);
    if (m && emit) ms_emit_add(em, out, claim && l == 0, v, (uint32_t)(oe - ob), m);
}

// One workgroup per CU at most (up to 128 VGPRs): the dense scan's state
// for a window of edges then stays in registers; at the 64-VGPR limit of
// two workgroups per CU it spilled to scratch, and the spill traffic cost
// more than the lost occupancy.
// Workgroup state of one batched round.
struct MsShared {
    uint32_t units[kMaxGroups + 1];
    uint32_t push[kMaxGroups];
    uint32_t wc[kMaxGroups];
    unsigned long long tot[kMaxGroups];
    uint32_t emit[kMaxGroups];
    uint32_t found[kMaxGroups];
    uint32_t fdsum[kMaxGroups];
    MsEmitBuf eb[kRWaves];  // one next-list buffer per wavefront
};

// Group G's list for round r + 1 (a frontier above the dense threshold
// abandons it, except under forced push).
__device__ __forceinline__ QueueOut ms_next_list(const MsGroupDev& G, uint32_t r, int32_t force_dir) {
    QueueOut out;
    out.Q = G.Q[(r + 1) & 1];
    out.P = G.P[(r + 1) & 1];
    out.qcnt = &G.ctl[(r + 1) & 3u];
    out.qover = &G.ctl[4 + ((r + 1) & 3u)];
    out.qlimit = force_dir == 1 ? ~0ull : G.dense_thresh;
    out.tot = nullptr;
    return out;
}

// One round r for every group (workgroup-uniform); returns false when no
// group has a frontier in round r (every group has finished).
// kSparseWin: the one-launch-per-round kernel picks kMsWinSparse windows on
// sparse graphs; the persistent kernel keeps kMsWin (its registers are full).
template <bool kSparseWin>
__device__ __forceinline__ bool ms_round(const MsArgs& A, uint32_t r, MsShared& sh) {
    uint32_t* s_units = sh.units;
    uint32_t* s_push = sh.push;
    uint32_t* s_wc = sh.wc;
    unsigned long long* s_tot = sh.tot;
    uint32_t* s_emit = sh.emit;
    uint32_t* s_found = sh.found;
    uint32_t* s_fdsum = sh.fdsum;
    const int l = lane_id();
    const int wib = threadIdx.x / kWave;
    const uint32_t nwaves = gridDim.x * kRWaves;
    const uint32_t gwave = blockIdx.x * kRWaves + wib;
    const int NG = A.ngroups;
    // totals of round r per group (wavefront gi reads group gi)
    for (int gi = wib; gi < NG; gi += kRWaves) {
        const unsigned long long t = spread_sum(ms_tot(A.groups[gi], r));
        // frontier size of round r-1: a dense round writes the sparse list
        // for round r+1 only while the frontier shrinks
        const unsigned long long tp = spread_sum(ms_tot(A.groups[gi], r + 3));
        if (l == 0) {
            s_tot[gi] = t;
            s_emit[gi] = (r > 0 && (uint32_t)(t >> 32) < (uint32_t)(tp >> 32)) ? 1u : 0u;
        }
    }
    if (threadIdx.x < (unsigned)NG) {
        s_found[threadIdx.x] = 0;
        s_fdsum[threadIdx.x] = 0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        // per-group direction and work units, prefix over groups
        uint32_t acc = 0;
        for (int gi = 0; gi < NG; ++gi) {
            const MsGroupDev& G = A.groups[gi];
            unsigned long long t = s_tot[gi];
            if (G.narrow && r > kNarrowRounds && (t >> 32) != 0ull) {
                // the 8-bit round field is full: the group stops here and
                // the host runs the call again with 8-byte entries
                t = 0ull;
                s_tot[gi] = 0ull;
                if (blockIdx.x == 0) *A.ovf |= 1ull << gi;
            }
            const uint32_t cnt = (uint32_t)(t >> 32), edges = (uint32_t)t;
            const bool qvalid = G.ctl[4 + (r & 3u)] == 0ull;
            bool push;
            if (A.force_dir == 1) push = true;
            else if (A.force_dir == 2) push = false;
            else push = qvalid && (uint64_t)cnt + edges <= G.dense_thresh;
            if (A.force_dir == 1 && !qvalid) push = false;
            s_push[gi] = push ? 1u : 0u;
            uint32_t units = 0;
            if (cnt) {
                if (push) {
                    const uint32_t wc = wave_chunk(edges, nwaves, A.chunk_cap);
                    s_wc[gi] = wc;
                    // the frontier itself must also be folded: one unit at least
                    units = max(1u, (edges + wc - 1) / wc);
                } else {
                    units = G.nplan;
                }
            }
            s_units[gi] = acc;
            acc += units;
            if (blockIdx.x == 0 && A.log && r < 4096) A.log[r * kMaxGroups + gi] = cnt ? (push ? 1u : 2u) : 0u;
        }
        s_units[NG] = acc;
    }
    __syncthreads();
    // clear slots of round r+2 and the frontier buffer round r+1 will write
    if (blockIdx.x == 0) {
        for (int gi = 0; gi < NG; ++gi) {
            if (threadIdx.x < kSpread) ms_tot(A.groups[gi], r + 2)[threadIdx.x * kSpreadStride] = 0ull;
            if (threadIdx.x == 0) {
                A.groups[gi].ctl[(r + 2) & 3u] = 0ull;
                A.groups[gi].ctl[4 + ((r + 2) & 3u)] = 0ull;
                if (!s_push[gi] && !s_emit[gi]) A.groups[gi].ctl[4 + ((r + 1) & 3u)] = 1ull;
            }
        }
    }
    for (int gi = 0; gi < NG; ++gi) {
        const MsGroupDev& G = A.groups[gi];
        const unsigned long long t = s_tot[gi];
        if ((t >> 32) == 0) continue;
        unsigned long long* Fclr = G.F[(r + 2) % 3];
        for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < G.n;
             v += (int64_t)gridDim.x * blockDim.x)
            Fclr[v] = 0ull;
        if (s_push[gi]) {
            // fold the frontier list into VM
            const uint32_t cnt = (uint32_t)(t >> 32);
            const uint32_t* Qc = G.Q[r & 1];
            const unsigned long long* Fc = G.F[r % 3];
            for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < cnt;
                 i += gridDim.x * blockDim.x) {
                const uint32_t u = Qc[i];
                G.VM[u] |= Fc[u];
            }
        }
    }
    const uint32_t total = s_units[NG];
    int gi = 0;
    uint32_t found = 0, dsum = 0;
    // this wavefront's buffered next-list entries belong to group egi
    MsEmitter em;
    em.b = &sh.eb[wib];
    em.n = 0u;
    int egi = -1;
    for (uint32_t unit = gwave; unit < total; unit += nwaves) {
        while (unit >= s_units[gi + 1]) ++gi;
        const MsGroupDev& G = A.groups[gi];
        const unsigned long long t = s_tot[gi];
        const uint32_t cnt = (uint32_t)(t >> 32), edges = (uint32_t)t;
        const QueueOut out = ms_next_list(G, r, A.force_dir);
        const unsigned long long* Fc = G.F[r % 3];
        unsigned long long* Fn = G.F[(r + 1) % 3];
        const uint32_t local = unit - s_units[gi];
        uint32_t f0 = 0, d0 = 0;
        if (s_push[gi] || s_emit[gi]) {
            // the buffered entries belong to one group's list
            if (egi != gi) {
                if (egi >= 0) ms_emit_flush(em, ms_next_list(A.groups[egi], r, A.force_dir));
                egi = gi;
            }
        }
        if (s_push[gi]) {
            if (edges) {
                MsPushPolicy pol{&G, Fc, Fn, &out, &em, r + 1u, 0u, 0u};
                const uint32_t wc = s_wc[gi];
                const uint32_t eb = local * wc;
                expand_range(G.Q[r & 1], G.P[r & 1], cnt, edges, G.off, eb, min(edges, eb + wc),
                             pol);
                f0 = pol.found;
                d0 = pol.dsum;
            }
        } else {
            const uint4 it = G.plan[local];
            const bool emit = s_emit[gi] != 0;
            if (it.z != kPlanHub)
                ms_pull_piece(G, r, it, Fc, Fn, em, out, emit, f0, d0);
            else if (kSparseWin && G.m <= 8ull * (uint64_t)G.n)
                ms_pull_run<kMsWinSparse>(G, r, it, Fc, Fn, em, out, emit, f0, d0);
            else
                ms_pull_run<kMsWin>(G, r, it, Fc, Fn, em, out, emit, f0, d0);
        }
        f0 = wave_sum(f0);
        d0 = wave_sum(d0);
        if (l == 0 && f0) {
            atomicAdd(&s_found[gi], f0);
            atomicAdd(&s_fdsum[gi], d0);
        }
    }
    if (egi >= 0) ms_emit_flush(em, ms_next_list(A.groups[egi], r, A.force_dir));
    __syncthreads();
    if (threadIdx.x < (unsigned)NG && s_found[threadIdx.x]) {
        const MsGroupDev& G = A.groups[threadIdx.x];
        atomicAdd(&ms_tot(G, r + 1)[(blockIdx.x % kSpread) * kSpreadStride],
                  ((unsigned long long)s_found[threadIdx.x] << 32) | s_fdsum[threadIdx.x]);
    }
    bool any = false;
    for (int g = 0; g < NG; ++g) any |= (s_tot[g] >> 32) != 0ull;
    return any;
}

__global__ __launch_bounds__(kRBlock, 1) void ms_round_kernel(MsArgs A, uint32_t r) {
    __shared__ MsShared sh;
    (void)ms_round<true>(A, r, sh);
}

// Every round of every group in one cooperative launch, a grid barrier
// between rounds; groups drop out as their frontiers empty and the kernel
// ends at the first round in which no group has a frontier (its number goes
// to bar[kBarUser]), after max_rounds, or when a barrier wait gave up (the
// abort word tells the host, which then runs the rounds one launch each).
__global__ __launch_bounds__(kRBlock, 1) void ms_persistent_kernel(MsArgs A, uint32_t* bar,
                                                                  uint32_t max_rounds) {
    __shared__ MsShared sh;
    __shared__ DieInfo di;
    if (!bar_census(bar, di)) return;
    uint32_t r = 0;
    for (; r < max_rounds; ++r) {
        if (!ms_round<false>(A, r, sh)) break;
        if (!grid_barrier(bar, di, r + 1)) return;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) bar[kBarUser] = r;
}

// Zeroes a grid-barrier area (kBarWords words).
__global__ void ms_bar_clear_kernel(uint32_t* bar) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < kBarWords; i += gridDim.x * blockDim.x)
        bar[i] = 0u;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
static size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t ms_group_bytes(int64_t n, int64_t k) {
    return 4 * al256((size_t)n * 8) + 4 * al256((size_t)(n + 64) * 4) +
           al256((8 + 4 * kSpread * kSpreadStride) * 8) + 2 * al256(64 * 8) + al256(64 * 4) +
           al256((size_t)n * (size_t)k * 8);
}

// Packs queries on the same graph 64 to a group (in submission order).
static std::vector<std::vector<int>> ms_plan(const std::vector<MsQuery>& qs) {
    std::vector<gbgpu_graph> order;
    std::vector<std::vector<int>> byg;
    for (int i = 0; i < (int)qs.size(); ++i) {
        int gi = -1;
        for (int j = 0; j < (int)order.size(); ++j)
            if (order[j] == qs[i].g) gi = j;
        if (gi < 0) {
            order.push_back(qs[i].g);
            byg.emplace_back();
            gi = (int)order.size() - 1;
        }
        byg[gi].push_back(i);
    }
    std::vector<std::vector<int>> groups;
    for (auto& v : byg)
        for (size_t b = 0; b < v.size(); b += 64)
            groups.emplace_back(v.begin() + b, v.begin() + std::min(v.size(), b + 64));
    return groups;
}

static size_t ms_header_bytes(int NG) {
    return al256(sizeof(MsGroupDev) * NG) + al256((size_t)NG * 64 * 4) +
           al256(4096 * kMaxGroups * 4) + al256((size_t)kBarWords * 4) + al256(8);
}

// Device bytes needed to run `groups` (at most kMaxGroups) together.
static size_t ms_chunk_bytes(const std::vector<MsQuery>& qs,
                             const std::vector<std::vector<int>>& groups, size_t g0, int NG) {
    size_t bytes = ms_header_bytes(NG);
    for (int i = 0; i < NG; ++i)
        bytes += ms_group_bytes(qs[groups[g0 + i][0]].g->n, (int64_t)groups[g0 + i].size());
    return bytes;
}

size_t ms_query_bytes(int64_t n, int64_t k) { return ms_header_bytes(1) + ms_group_bytes(n, k); }

size_t ms_pin_bytes() { return (size_t)kMaxGroups * kSpread * kSpreadStride * 8; }

// Runs every round of the groups in A (initialised and seeded on `stream`)
// in one cooperative launch of at most `grid` workgroups (fewer if that many
// cannot all be resident), then waits for it.  *done is false when the
// launch was refused or a barrier wait gave up: the groups' state is then
// partial and the caller starts them again.  *rounds is the first round in
// which no group had a frontier.  `hp` is pinned host memory (two words).
static int ms_run_persistent(const MsArgs& A, uint32_t* dbar, int grid, gbgpu_graph g,
                             int64_t max_rounds, unsigned long long* hp, hipStream_t stream,
                             bool* done, uint32_t* rounds) {
    *done = false;
    int coop = 0;
    if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, g->device) !=
            hipSuccess || !coop)
        return GBGPU_OK;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, reinterpret_cast<const void*>(ms_persistent_kernel), kRBlock, 0) !=
            hipSuccess || per_cu < 1)
        return GBGPU_OK;
    const int pgrid = std::max(1, std::min(grid, per_cu * g->num_cus));
    hipLaunchKernelGGL(ms_bar_clear_kernel, dim3(4), dim3(kBlock), 0, stream, dbar);
    GB_HIP(hipGetLastError());
    MsArgs ka = A;
    uint32_t* bar = dbar;
    uint32_t maxr = (uint32_t)std::min<int64_t>(max_rounds, 0xFFFFFFFFll);
    void* args[] = {&ka, &bar, &maxr};
    if (hipLaunchCooperativeKernel(reinterpret_cast<const void*>(ms_persistent_kernel),
                                   dim3(pgrid), dim3(kRBlock), args, 0, stream) != hipSuccess) {
        (void)hipGetLastError();  // refused: the caller runs one launch per round
        return GBGPU_OK;
    }
    uint32_t* h = reinterpret_cast<uint32_t*>(hp);
    GB_HIP(hipMemcpyAsync(h, dbar + kBarAbort, 4, hipMemcpyDeviceToHost, stream));
    GB_HIP(hipMemcpyAsync(h + 1, dbar + kBarUser, 4, hipMemcpyDeviceToHost, stream));
    GB_HIP(hipStreamSynchronize(stream));
    if (h[0] != 0u) return GBGPU_OK;
    if ((int64_t)h[1] >= max_rounds) return set_error(GBGPU_E_HIP, "batched BFS did not terminate");
    *rounds = h[1];
    *done = true;
    return GBGPU_OK;
}

// Runs groups[g0 .. g0+NG) in one launch per round (or, when opts.persistent
// is 1 and no hook is given, every round in one launch), with `mem` holding
// ms_chunk_bytes() bytes of device memory and `pin` ms_pin_bytes() of pinned
// host memory.
// With a join hook (one group only) the group's staging holds kcap sources
// and the hook is asked at every round boundary the host sees (every 4
// launches) for queries to add: up to kcap - kused of them join before the
// next round.
static int ms_run_chunk(const std::vector<MsQuery>& qs, const std::vector<std::vector<int>>& groups,
                        size_t gb0, int NG, void* mem, void* pin, const gbgpu_opts& o,
                        hipStream_t stream, int* rounds_out, int* launches_out,
                        uint32_t kcap = 0, const MsJoinHook* hook = nullptr) {
    const bool joinable = hook != nullptr && NG == 1;
    char* p = (char*)mem;
    MsGroupDev* dgroups = (MsGroupDev*)p; p += al256(sizeof(MsGroupDev) * NG);
    uint32_t* dsrcs = (uint32_t*)p; p += al256((size_t)NG * 64 * 4);
    uint32_t* dlog = (uint32_t*)p; p += al256(4096 * kMaxGroups * 4);
    uint32_t* dbar = (uint32_t*)p; p += al256((size_t)kBarWords * 4);
    unsigned long long* dovf = (unsigned long long*)p; p += al256(8);
    std::vector<MsGroupDev> hg(NG);
    std::vector<uint32_t> hsrc((size_t)NG * 64, 0);
    std::vector<int32_t*> rowsD((size_t)NG * 64, nullptr), rowsP((size_t)NG * 64, nullptr);
    int64_t maxn = 0;
    for (int i = 0; i < NG; ++i) {
        const auto& gq = groups[gb0 + i];
        gbgpu_graph g = qs[gq[0]].g;
        MsGroupDev& G = hg[i];
        const int64_t n = g->n;
        maxn = std::max(maxn, n);
        G.off = g->off;
        G.nbr = g->nbr;
        G.deg = g->deg;
        G.n = n;
        G.dense_thresh = (uint64_t)g->m / (uint64_t)o.tau;
        G.m = (uint64_t)g->m;
        G.kmask = gq.size() == 64 ? ~0ull : ((1ull << gq.size()) - 1ull);
        GB_TRY(ensure_pull_plan(g));
        G.plan = g->plan;
        G.nplan = g->nplan;
        G.VM = (unsigned long long*)p; p += al256((size_t)n * 8);
        for (int b = 0; b < 3; ++b) { G.F[b] = (unsigned long long*)p; p += al256((size_t)n * 8); }
        for (int b = 0; b < 2; ++b) { G.Q[b] = (uint32_t*)p; p += al256((size_t)(n + 64) * 4); }
        for (int b = 0; b < 2; ++b) { G.P[b] = (uint32_t*)p; p += al256((size_t)(n + 64) * 4); }
        G.ctl = (unsigned long long*)p; p += al256((8 + 4 * kSpread * kSpreadStride) * 8);
        G.drow = (int32_t* const*)p; p += al256(64 * 8);
        G.prow = (int32_t* const*)p; p += al256(64 * 8);
        G.start = (uint32_t*)p; p += al256(64 * 4);
        G.k = (uint32_t)std::max<size_t>(gq.size(), joinable ? kcap : 0u);
        G.kused = (uint32_t)gq.size();
        // 4-byte entries where a parent fits in 24 bits, no source joins
        // later (the round field then counts from 0) and no search has shown
        // the graph deeper than the field; room for 8-byte entries either
        // way, for the rerun after a round overflow
        G.narrow = (!joinable && n <= ((int64_t)1 << 24) &&
                    g->depth.load(std::memory_order_relaxed) <= (int32_t)kNarrowRounds)
                       ? 1u : 0u;
        G.E = (void*)p; p += al256((size_t)n * G.k * 8);
        for (size_t j = 0; j < gq.size(); ++j) {
            hsrc[(size_t)i * 64 + j] = (uint32_t)qs[gq[j]].src;
            rowsD[(size_t)i * 64 + j] = qs[gq[j]].dist;
            rowsP[(size_t)i * 64 + j] = qs[gq[j]].parent;
        }
        GB_HIP(hipMemcpyAsync((void*)G.drow, &rowsD[(size_t)i * 64], 64 * 8, hipMemcpyHostToDevice, stream));
        GB_HIP(hipMemcpyAsync((void*)G.prow, &rowsP[(size_t)i * 64], 64 * 8, hipMemcpyHostToDevice, stream));
    }
    GB_HIP(hipMemcpyAsync(dgroups, hg.data(), sizeof(MsGroupDev) * NG, hipMemcpyHostToDevice, stream));
    GB_HIP(hipMemcpyAsync(dsrcs, hsrc.data(), (size_t)NG * 64 * 4, hipMemcpyHostToDevice, stream));
    auto init_groups = [&]() {
        for (int i = 0; i < NG; ++i) {
            const int k = (int)groups[gb0 + i].size();
            const int ig =
                (int)std::min<int64_t>(std::max<int64_t>((hg[i].n + kBlock - 1) / kBlock, 1), 4096);
            hipLaunchKernelGGL(ms_init_kernel, dim3(ig), dim3(kBlock), 0, stream, dgroups, i,
                               dsrcs + (size_t)i * 64, k);
            hipLaunchKernelGGL(ms_seed_kernel, dim3(1), dim3(64), 0, stream, dgroups, i,
                               dsrcs + (size_t)i * 64, k, i == 0 ? dovf : nullptr);
        }
        return hipGetLastError();
    };
    MsArgs A;
    A.groups = dgroups;
    A.ovf = dovf;
    A.ngroups = NG;
    A.force_dir = o.force_direction == 3 ? 0 : o.force_direction;
    A.light = o.pull_light;
    A.chunk_cap = (uint32_t)o.wave_chunk;
    A.log = dlog;
    int64_t work = 0;
    for (int i = 0; i < NG; ++i) work += std::max<int64_t>(hg[i].n / 64, 1);
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((work + kRWaves - 1) / kRWaves, o.grid));
    unsigned long long* hp = (unsigned long long*)pin;
    bool narrow = false;
    for (int i = 0; i < NG; ++i) narrow |= hg[i].narrow != 0u;
    uint32_t r = 0;
    uint32_t kused = hg[0].kused;
    // every round of every group, from the sources
    auto run_rounds = [&]() -> int {
        GB_HIP(init_groups());
        r = 0;
        int64_t round_limit = maxn + 2;
        bool done = false;
        if (o.persistent > 0 && !joinable) {
            // every round in one cooperative launch; if the launch is refused or
            // a barrier wait gave up, the groups start again one launch per round
            GB_TRY(ms_run_persistent(A, dbar, grid, qs[groups[gb0][0]].g, round_limit, hp, stream,
                                     &done, &r));
            if (done) {
                *launches_out += 1;
            } else {
                r = 0;
                GB_HIP(init_groups());
            }
        }
        // rounds here take milliseconds: a completion check per batch is cheap;
        // a group that admits arrivals checks every 4 rounds
        int K = joinable ? 4 : 8;
        while (!done) {
            for (int i = 0; i < K; ++i)
                hipLaunchKernelGGL(ms_round_kernel, dim3(grid), dim3(kRBlock), 0, stream, A, r + i);
            GB_HIP(hipGetLastError());
            r += (uint32_t)K;
            *launches_out += K;
            for (int i = 0; i < NG; ++i)
                GB_HIP(hipMemcpyAsync(hp + (size_t)i * kSpread * kSpreadStride,
                                      hg[i].ctl + 8 + (size_t)(r & 3u) * kSpread * kSpreadStride,
                                      kSpread * kSpreadStride * 8, hipMemcpyDeviceToHost, stream));
            GB_HIP(hipStreamSynchronize(stream));
            bool active = false;
            for (int i = 0; i < NG && !active; ++i) {
                unsigned long long t = 0;
                for (int c = 0; c < kSpread; ++c)
                    t += hp[(size_t)i * kSpread * kSpreadStride + c * kSpreadStride];
                active = (t >> 32) != 0;
            }
            if (joinable && kused < hg[0].k) {
                // round boundary r: queries waiting for this graph join the group
                std::vector<MsQuery> add;
                (*hook)(r, (int)(hg[0].k - kused), !active, &add);
                if (!add.empty()) {
                    const uint32_t nadd = (uint32_t)std::min<size_t>(add.size(), hg[0].k - kused);
                    for (uint32_t i = 0; i < nadd; ++i) {
                        hsrc[kused + i] = (uint32_t)add[i].src;
                        rowsD[kused + i] = add[i].dist;
                        rowsP[kused + i] = add[i].parent;
                    }
                    GB_HIP(hipMemcpyAsync((void*)(hg[0].drow + kused), &rowsD[kused], nadd * 8,
                                          hipMemcpyHostToDevice, stream));
                    GB_HIP(hipMemcpyAsync((void*)(hg[0].prow + kused), &rowsP[kused], nadd * 8,
                                          hipMemcpyHostToDevice, stream));
                    GB_HIP(hipMemcpyAsync(dsrcs + kused, &hsrc[kused], nadd * 4,
                                          hipMemcpyHostToDevice, stream));
                    if (!active) {
                        const int cg = (int)std::min<int64_t>(
                            std::max<int64_t>((hg[0].n + kBlock - 1) / kBlock, 1), 4096);
                        hipLaunchKernelGGL(ms_clear_frontiers_kernel, dim3(cg), dim3(kBlock), 0,
                                           stream, dgroups, 0);
                    }
                    hipLaunchKernelGGL(ms_join_kernel, dim3(1), dim3(64), 0, stream, dgroups, 0, r,
                                       dsrcs + kused, kused, nadd);
                    GB_HIP(hipGetLastError());
                    kused += nadd;
                    round_limit = (int64_t)r + maxn + 2;
                    active = true;
                }
            }
            if (!active) break;
            if ((int64_t)r > round_limit)
                return set_error(GBGPU_E_HIP, "batched BFS did not terminate");
            if (!joinable) K = std::min(K * 2, 512);
        }
        return GBGPU_OK;
    };
    GB_TRY(run_rounds());
    if (narrow) {
        unsigned long long ovf = 0;
        GB_HIP(hipMemcpyAsync(&ovf, dovf, 8, hipMemcpyDeviceToHost, stream));
        GB_HIP(hipStreamSynchronize(stream));
        if (ovf) {
            // a search ran past round kNarrowRounds: its graph is marked that
            // deep (later calls start with 8-byte entries), and every group
            // runs again with 8-byte entries
            for (int i = 0; i < NG; ++i) {
                if ((ovf >> i) & 1ull) {
                    gbgpu_graph g = qs[groups[gb0 + i][0]].g;
                    int32_t d = g->depth.load(std::memory_order_relaxed);
                    while (d <= (int32_t)kNarrowRounds &&
                           !g->depth.compare_exchange_weak(d, (int32_t)kNarrowRounds + 1,
                                                           std::memory_order_relaxed)) {
                    }
                }
                hg[i].narrow = 0u;
            }
            GB_HIP(hipMemcpyAsync(dgroups, hg.data(), sizeof(MsGroupDev) * NG,
                                  hipMemcpyHostToDevice, stream));
            GB_TRY(run_rounds());
        }
    }
    for (int i = 0; i < NG; ++i) {
        const int tg = (int)std::min<int64_t>(std::max<int64_t>((hg[i].n + 63) / 64, 1), 8192);
        hipLaunchKernelGGL(ms_transpose_kernel, dim3(tg), dim3(kBlock), 0, stream, dgroups, i);
    }
    GB_HIP(hipGetLastError());
    GB_HIP(hipStreamSynchronize(stream));
    *rounds_out = std::max<int>(*rounds_out, (int)r);
    return GBGPU_OK;
}

// Runs every query with a workspace that grows as needed.
int run_ms(const std::vector<MsQuery>& qs, const gbgpu_opts& o, gbgpu_stats* st,
           hipStream_t stream, MultiWs** wsp) {
    const double t0 = now_ms();
    const auto groups = ms_plan(qs);
    int launches = 0, rounds = 0;
    for (size_t gb0 = 0; gb0 < groups.size(); gb0 += kMaxGroups) {
        const int NG = (int)std::min<size_t>(kMaxGroups, groups.size() - gb0);
        const size_t bytes = ms_chunk_bytes(qs, groups, gb0, NG);
        MultiWs*& w = *wsp;
        if (!w || w->bytes < bytes) {
            free_multi_ws(w);
            w = new MultiWs();
            hipError_t e = hipMalloc(&w->block, bytes);
            if (e != hipSuccess) {
                delete w;
                w = nullptr;
                return set_error(GBGPU_E_NOMEM, "batched BFS workspace of %zu bytes: %s", bytes,
                                 hipGetErrorString(e));
            }
            w->bytes = bytes;
            if (hipHostMalloc(&w->host_pin, ms_pin_bytes(), hipHostMallocDefault) != hipSuccess)
                return set_error(GBGPU_E_HIP, "pinned buffer allocation failed");
        }
        GB_TRY(ms_run_chunk(qs, groups, gb0, NG, w->block, w->host_pin, o, stream, &rounds, &launches));
    }
    if (st) {
        memset(st, 0, sizeof(*st));
        st->launches = launches;
        st->rounds = rounds;
        st->wall_ms = now_ms() - t0;
    }
    return GBGPU_OK;
}

// One group (<= 64 queries on one graph) with caller-provided memory
// (ms_query_bytes(n, max(k, kcap)) device bytes, ms_pin_bytes() pinned
// bytes); with a hook, up to kcap - k more queries may join it at round
// boundaries.
int run_ms_group_mem(const std::vector<MsQuery>& qs, void* mem, void* pin, const gbgpu_opts& o,
                     hipStream_t stream, int* rounds, uint32_t kcap, const MsJoinHook* hook) {
    std::vector<std::vector<int>> groups(1);
    for (int i = 0; i < (int)qs.size(); ++i) groups[0].push_back(i);
    int launches = 0;
    *rounds = 0;
    return ms_run_chunk(qs, groups, 0, 1, mem, pin, o, stream, rounds, &launches, kcap, hook);
}

}  // namespace gb

using namespace gb;

extern "C" {

int gbgpu_bfs_multi(gbgpu_graph g, const int32_t* srcs, int32_t k, int32_t* dist, int32_t* parent,
                    const gbgpu_opts* o, gbgpu_stats* st, void* stream) {
    if (!g) return set_error(GBGPU_E_INVALID, "graph is NULL");
    if (!srcs || k < 1) return set_error(GBGPU_E_INVALID, "need k >= 1 sources");
    if (!dist || !parent) return set_error(GBGPU_E_INVALID, "dist/parent is NULL");
    for (int i = 0; i < k; ++i)
        if (srcs[i] < 0 || srcs[i] >= g->n)
            return set_error(GBGPU_E_INVALID, "source %d = %d out of range", i, srcs[i]);
    gbgpu_opts opt = resolve_opts(o);
    std::vector<MsQuery> qs((size_t)k);
    for (int i = 0; i < k; ++i)
        qs[i] = MsQuery{g, srcs[i], dist + (size_t)i * g->n, parent + (size_t)i * g->n};
    std::lock_guard<std::mutex> lk(g->mu);
    return run_ms(qs, opt, st, (hipStream_t)stream, &g->multi);
}

// Diagnostic: a packed group of srcs[0 .. k0) joined by srcs[k0 .. k0+k1)
// at the first round boundary at or after join_round (or when the group runs
// out of work first); rows of dist / parent with stride n.
int gbgpu_debug_bfs_join(gbgpu_graph g, const int32_t* srcs, int32_t k0, int32_t k1,
                         int32_t join_round, int32_t* dist, int32_t* parent, void* stream) {
    if (!g || !srcs || !dist || !parent) return set_error(GBGPU_E_INVALID, "bad argument");
    if (k0 < 1 || k1 < 0 || k0 + k1 > 64 || join_round < 0)
        return set_error(GBGPU_E_INVALID, "need k0 >= 1, k1 >= 0, k0 + k1 <= 64");
    for (int i = 0; i < k0 + k1; ++i)
        if (srcs[i] < 0 || srcs[i] >= g->n)
            return set_error(GBGPU_E_INVALID, "source %d = %d out of range", i, srcs[i]);
    gbgpu_opts opt = resolve_opts(nullptr);
    hipStream_t s = (hipStream_t)stream;
    std::lock_guard<std::mutex> lk(g->mu);
    GB_TRY(ensure_pull_plan(g));
    const size_t bytes = ms_query_bytes(g->n, 64);
    void* mem = nullptr;
    void* pin = nullptr;
    if (hipMalloc(&mem, bytes) != hipSuccess)
        return set_error(GBGPU_E_NOMEM, "join test workspace of %zu bytes", bytes);
    if (hipHostMalloc(&pin, ms_pin_bytes(), hipHostMallocDefault) != hipSuccess) {
        (void)hipFree(mem);
        return set_error(GBGPU_E_NOMEM, "pinned buffer allocation failed");
    }
    std::vector<MsQuery> qs, later;
    for (int i = 0; i < k0 + k1; ++i)
        (i < k0 ? qs : later)
            .push_back(MsQuery{g, srcs[i], dist + (size_t)i * g->n, parent + (size_t)i * g->n});
    bool joined = later.empty();
    MsJoinHook hook = [&](uint32_t r, int room, bool idle, std::vector<MsQuery>* add) {
        if (joined || ((int32_t)r < join_round && !idle) || room < (int)later.size()) return;
        *add = later;
        joined = true;
    };
    int rounds = 0;
    const int st = run_ms_group_mem(qs, mem, pin, opt, s, &rounds, 64u, &hook);
    (void)hipStreamSynchronize(s);
    (void)hipFree(mem);
    (void)hipHostFree(pin);
    if (st != GBGPU_OK) return st;
    if (!joined) return set_error(GBGPU_E_HIP, "the joining sources were never admitted");
    return GBGPU_OK;
}

static std::mutex g_batch_mu;
static MultiWs* g_batch_ws = nullptr;

int gbgpu_bfs_batch(const gbgpu_graph* graphs, const int32_t* srcs, int32_t nq,
                    int32_t* const* dists, int32_t* const* parents, const gbgpu_opts* o,
                    gbgpu_stats* st, void* stream) {
    if (!graphs || !srcs || !dists || !parents || nq < 1)
        return set_error(GBGPU_E_INVALID, "bad batch arguments");
    std::vector<MsQuery> qs((size_t)nq);
    for (int i = 0; i < nq; ++i) {
        if (!graphs[i]) return set_error(GBGPU_E_INVALID, "graph %d is NULL", i);
        if (srcs[i] < 0 || srcs[i] >= graphs[i]->n)
            return set_error(GBGPU_E_INVALID, "query %d: source out of range", i);
        if (!dists[i] || !parents[i]) return set_error(GBGPU_E_INVALID, "query %d: NULL output", i);
        qs[i] = MsQuery{graphs[i], srcs[i], dists[i], parents[i]};
    }
    gbgpu_opts opt = resolve_opts(o);
    std::lock_guard<std::mutex> lk(g_batch_mu);
    return run_ms(qs, opt, st, (hipStream_t)stream, &g_batch_ws);
}

}  // extern "C"
