// Batched BFS: many sources, possibly on many graphs, in one launch per round.
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
//     OR-ed into F_{r+1}[v] and every such bit j takes atomicMin(parent_j[v], u);
//   pull (dense): every vertex with unseen bits scans its ascending list; the
//     first neighbour u that carries bit j in F_r becomes parent_j[v] (a
//     wavefront prefix-OR finds first contributors when a whole wavefront
//     scans one list), with early exit once every unseen bit is found.
// Both rules give parent_j[v] = min{u in N(v) : D_j[u] = D_j[v] - 1}, so each
// row equals the single-source BFS from source j.  Distances are written when
// a vertex's bits enter the frontier: D_j[v] = r for the bits of F_r[v].
// Groups finish independently; a finished group costs nothing.

#include "common.h"
#include "emit.h"

namespace gb {

constexpr int kMaxGroups = 64;

struct MsGroupDev {
    const int64_t* off;
    const int32_t* nbr;
    const uint32_t* deg;
    int64_t n;
    uint64_t dense_thresh;
    unsigned long long kmask;   // bits of the sources in this group
    unsigned long long* VM;     // n
    unsigned long long* F[3];   // n each
    uint32_t* Q[2];             // n + 64 each
    uint32_t* P[2];
    unsigned long long* ctl;    // [0..3] qcnt, [4..7] qover, then 4 x kSpread x kSpreadStride totals
    int32_t* const* drow;       // 64 row pointers (dist), device array
    int32_t* const* prow;       // 64 row pointers (parent), device array
};

struct MsArgs {
    MsGroupDev* groups;
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
    for (int j = 0; j < k; ++j) {
        int32_t* dr = G.drow[j];
        int32_t* pr = G.prow[j];
        for (int64_t v = tid; v < G.n; v += stride) {
            dr[v] = INT32_MAX;
            pr[v] = v == (int64_t)srcs[j] ? (int32_t)srcs[j] : -1;
        }
    }
    for (int64_t i = tid; i < 8 + 4 * kSpread * kSpreadStride; i += stride) G.ctl[i] = 0ull;
}

// After init: frontier F_0 = source bits, list Q_0 = distinct sources.
__global__ void ms_seed_kernel(MsGroupDev* groups, int32_t gi, const uint32_t* srcs, int32_t k) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const MsGroupDev G = groups[gi];
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
    }
    G.ctl[0] = ((unsigned long long)cnt << 32) | edges;  // qcnt slot 0
    ms_tot(G, 0)[0] = ((unsigned long long)cnt << 32) | edges;
}

struct MsPushPolicy {
    const MsGroupDev* G;
    const unsigned long long* Fc;
    unsigned long long* Fn;
    const QueueOut* out;
    uint32_t found;
    uint32_t dsum;
    static constexpr bool kSkipDead = false;

    __device__ __forceinline__ uint32_t aux(uint32_t) const { return 1u; }

    __device__ __forceinline__ void edge(bool act, uint32_t u, uint32_t, int64_t e) {
        bool claim = false;
        uint32_t v = 0, dv = 0;
        if (act) {
            v = (uint32_t)G->nbr[e];
            const unsigned long long seen = G->VM[v] | Fc[v];
            const unsigned long long cand = Fc[u] & G->kmask & ~seen;
            if (cand) {
                const unsigned long long old = atomicOr(&Fn[v], cand);
                claim = old == 0ull;
                unsigned long long bits = cand;
                while (bits) {
                    const int j = __ffsll((long long)bits) - 1;
                    bits &= bits - 1;
                    uint32_t* pp = (uint32_t*)G->prow[j] + v;
                    if (u < *pp) atomicMin(pp, u);
                }
                if (claim) dv = G->deg[v];
            }
        }
        const uint64_t m = ballot(claim);
        if (m) {
            wave_direct_emit(claim, v, dv, m, *out);
            if (claim) {
                found += 1;
                dsum += dv;
            }
        }
    }
    __device__ __forceinline__ void window_done() {}
};

// Dense processing of 64 consecutive vertices of one group by one wavefront.
__device__ __forceinline__ void ms_pull_group(const MsGroupDev& G, uint32_t r, int64_t vg,
                                              const unsigned long long* __restrict__ Fc,
                                              unsigned long long* Fn, const QueueOut& out,
                                              bool emit, int light, uint32_t& found,
                                              uint32_t& dsum) {
    const int l = lane_id();
    const int64_t v64 = 64 * vg + l;
    const bool inb = v64 < G.n;
    const uint32_t v = (uint32_t)v64;
    unsigned long long need = 0ull;
    int64_t s = 0, e = 0;
    if (inb) {
        const unsigned long long f = Fc[v];
        unsigned long long vm = G.VM[v];
        if (f) {
            // v's bits entered the frontier in round r: record the distance
            vm |= f;
            G.VM[v] = vm;
            unsigned long long bits = f;
            while (bits) {
                const int j = __ffsll((long long)bits) - 1;
                bits &= bits - 1;
                G.drow[j][v] = (int32_t)r;
            }
        }
        need = G.kmask & ~vm;
        s = G.off[v];
        e = G.off[v + 1];
        if (s == e) need = 0ull;
    }
    unsigned long long acc = 0ull;
    int64_t k = s;
    const int64_t lim = min(e, s + (int64_t)light);
    // light phase: one lane per vertex, ascending order, stop when all
    // unseen bits are found
    while (need && acc != need && k < lim) {
        const uint32_t u = (uint32_t)G.nbr[k];
        const unsigned long long add = Fc[u] & need & ~acc;
        if (add) {
            acc |= add;
            unsigned long long bits = add;
            while (bits) {
                const int j = __ffsll((long long)bits) - 1;
                bits &= bits - 1;
                G.prow[j][v] = (int32_t)u;
            }
        }
        ++k;
    }
    // heavy phase: the whole wavefront scans the rest of one list 64 at a
    // time; a prefix OR over lanes gives each bit's first contributor
    uint64_t hm = ballot(need && acc != need && k < e);
    while (hm) {
        const int h = first_lane(hm);
        hm &= hm - 1;
        const int64_t hs = (int64_t)shfl64((uint64_t)k, h);
        const int64_t he = (int64_t)shfl64((uint64_t)e, h);
        const unsigned long long hneed = shfl64(need, h);
        unsigned long long hacc = shfl64(acc, h);
        const uint32_t hv = __shfl(v, h, 64);
        for (int64_t b = hs; b < he && hacc != hneed; b += 64) {
            const int64_t i = b + l;
            uint32_t u = 0;
            unsigned long long add = 0ull;
            if (i < he) {
                u = (uint32_t)G.nbr[i];
                add = Fc[u] & hneed & ~hacc;
            }
            const unsigned long long before = wave_excl_or64(add);
            unsigned long long first = add & ~before;
            while (first) {
                const int j = __ffsll((long long)first) - 1;
                first &= first - 1;
                G.prow[j][hv] = (int32_t)u;
            }
            unsigned long long all = add;
#pragma unroll
            for (int d = 32; d >= 1; d >>= 1) {
                const uint32_t lo = __shfl_xor((uint32_t)all, d, 64);
                const uint32_t hi = __shfl_xor((uint32_t)(all >> 32), d, 64);
                all |= ((unsigned long long)hi << 32) | lo;
            }
            hacc |= all;
        }
        if (l == h) acc = hacc;
    }
    if (inb) Fn[v] = acc;
    const bool got = acc != 0ull;
    const uint32_t dv = got ? (uint32_t)(e - s) : 0u;
    const uint64_t m = ballot(got);
    if (m) {
        if (emit) wave_direct_emit(got, v, dv, m, out);
        if (got) {
            found += 1;
            dsum += dv;
        }
    }
}

__global__ __launch_bounds__(kRBlock, 8) void ms_round_kernel(MsArgs A, uint32_t r) {
    __shared__ uint32_t s_units[kMaxGroups + 1];
    __shared__ uint32_t s_push[kMaxGroups];
    __shared__ uint32_t s_wc[kMaxGroups];
    __shared__ unsigned long long s_tot[kMaxGroups];
    __shared__ uint32_t s_emit[kMaxGroups];
    __shared__ uint32_t s_found[kMaxGroups];
    __shared__ uint32_t s_fdsum[kMaxGroups];
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
            const unsigned long long t = s_tot[gi];
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
                    units = (uint32_t)((G.n + 63) / 64);
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
            // fold the frontier list into VM and record distances
            const uint32_t cnt = (uint32_t)(t >> 32);
            const uint32_t* Qc = G.Q[r & 1];
            const unsigned long long* Fc = G.F[r % 3];
            for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < cnt;
                 i += gridDim.x * blockDim.x) {
                const uint32_t u = Qc[i];
                const unsigned long long f = Fc[u];
                G.VM[u] |= f;
                unsigned long long bits = f;
                while (bits) {
                    const int j = __ffsll((long long)bits) - 1;
                    bits &= bits - 1;
                    G.drow[j][u] = (int32_t)r;
                }
            }
        }
    }
    const uint32_t total = s_units[NG];
    int gi = 0;
    uint32_t found = 0, dsum = 0;
    for (uint32_t unit = gwave; unit < total; unit += nwaves) {
        while (unit >= s_units[gi + 1]) ++gi;
        const MsGroupDev& G = A.groups[gi];
        const unsigned long long t = s_tot[gi];
        const uint32_t cnt = (uint32_t)(t >> 32), edges = (uint32_t)t;
        QueueOut out;
        out.Q = G.Q[(r + 1) & 1];
        out.P = G.P[(r + 1) & 1];
        out.qcnt = &G.ctl[(r + 1) & 3u];
        out.qover = &G.ctl[4 + ((r + 1) & 3u)];
        out.qlimit = A.force_dir == 1 ? ~0ull : G.dense_thresh;
        out.tot = nullptr;
        const unsigned long long* Fc = G.F[r % 3];
        unsigned long long* Fn = G.F[(r + 1) % 3];
        const uint32_t local = unit - s_units[gi];
        uint32_t f0 = 0, d0 = 0;
        if (s_push[gi]) {
            if (edges) {
                MsPushPolicy pol{&G, Fc, Fn, &out, 0u, 0u};
                const uint32_t wc = s_wc[gi];
                const uint32_t eb = local * wc;
                expand_range(G.Q[r & 1], G.P[r & 1], cnt, edges, G.off, eb, min(edges, eb + wc),
                             pol);
                f0 = pol.found;
                d0 = pol.dsum;
            }
        } else {
            ms_pull_group(G, r, (int64_t)local, Fc, Fn, out, s_emit[gi] != 0, A.light, f0, d0);
        }
        f0 = wave_sum(f0);
        d0 = wave_sum(d0);
        if (l == 0 && f0) {
            atomicAdd(&s_found[gi], f0);
            atomicAdd(&s_fdsum[gi], d0);
        }
    }
    __syncthreads();
    if (threadIdx.x < (unsigned)NG && s_found[threadIdx.x]) {
        const MsGroupDev& G = A.groups[threadIdx.x];
        atomicAdd(&ms_tot(G, r + 1)[(blockIdx.x % kSpread) * kSpreadStride],
                  ((unsigned long long)s_found[threadIdx.x] << 32) | s_fdsum[threadIdx.x]);
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
static size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t ms_group_bytes(int64_t n) {
    return 4 * al256((size_t)n * 8) + 4 * al256((size_t)(n + 64) * 4) +
           al256((8 + 4 * kSpread * kSpreadStride) * 8) + 2 * al256(64 * 8) + al256(64 * 4);
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
           al256(4096 * kMaxGroups * 4);
}

// Device bytes needed to run `groups` (at most kMaxGroups) together.
static size_t ms_chunk_bytes(const std::vector<MsQuery>& qs,
                             const std::vector<std::vector<int>>& groups, size_t g0, int NG) {
    size_t bytes = ms_header_bytes(NG);
    for (int i = 0; i < NG; ++i) bytes += ms_group_bytes(qs[groups[g0 + i][0]].g->n);
    return bytes;
}

size_t ms_query_bytes(int64_t n) { return ms_header_bytes(1) + ms_group_bytes(n); }

size_t ms_pin_bytes() { return (size_t)kMaxGroups * kSpread * kSpreadStride * 8; }

// Runs groups[g0 .. g0+NG) in one launch per round, with `mem` holding
// ms_chunk_bytes() bytes of device memory and `pin` ms_pin_bytes() of pinned
// host memory.
static int ms_run_chunk(const std::vector<MsQuery>& qs, const std::vector<std::vector<int>>& groups,
                        size_t gb0, int NG, void* mem, void* pin, const gbgpu_opts& o,
                        hipStream_t stream, int* rounds_out, int* launches_out) {
    char* p = (char*)mem;
    MsGroupDev* dgroups = (MsGroupDev*)p; p += al256(sizeof(MsGroupDev) * NG);
    uint32_t* dsrcs = (uint32_t*)p; p += al256((size_t)NG * 64 * 4);
    uint32_t* dlog = (uint32_t*)p; p += al256(4096 * kMaxGroups * 4);
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
        G.kmask = gq.size() == 64 ? ~0ull : ((1ull << gq.size()) - 1ull);
        G.VM = (unsigned long long*)p; p += al256((size_t)n * 8);
        for (int b = 0; b < 3; ++b) { G.F[b] = (unsigned long long*)p; p += al256((size_t)n * 8); }
        for (int b = 0; b < 2; ++b) { G.Q[b] = (uint32_t*)p; p += al256((size_t)(n + 64) * 4); }
        for (int b = 0; b < 2; ++b) { G.P[b] = (uint32_t*)p; p += al256((size_t)(n + 64) * 4); }
        G.ctl = (unsigned long long*)p; p += al256((8 + 4 * kSpread * kSpreadStride) * 8);
        G.drow = (int32_t* const*)p; p += al256(64 * 8);
        G.prow = (int32_t* const*)p; p += al256(64 * 8);
        p += al256(64 * 4);
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
    for (int i = 0; i < NG; ++i) {
        const int k = (int)groups[gb0 + i].size();
        const int ig = (int)std::min<int64_t>(std::max<int64_t>((hg[i].n + kBlock - 1) / kBlock, 1), 4096);
        hipLaunchKernelGGL(ms_init_kernel, dim3(ig), dim3(kBlock), 0, stream, dgroups, i,
                           dsrcs + (size_t)i * 64, k);
        hipLaunchKernelGGL(ms_seed_kernel, dim3(1), dim3(64), 0, stream, dgroups, i,
                           dsrcs + (size_t)i * 64, k);
    }
    GB_HIP(hipGetLastError());
    MsArgs A;
    A.groups = dgroups;
    A.ngroups = NG;
    A.force_dir = o.force_direction == 3 ? 0 : o.force_direction;
    A.light = o.pull_light;
    A.chunk_cap = (uint32_t)o.wave_chunk;
    A.log = dlog;
    int64_t work = 0;
    for (int i = 0; i < NG; ++i) work += std::max<int64_t>(hg[i].n / 64, 1);
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((work + kRWaves - 1) / kRWaves, o.grid));
    uint32_t r = 0;
    int K = o.rounds_per_sync;
    unsigned long long* hp = (unsigned long long*)pin;
    for (;;) {
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
            for (int c = 0; c < kSpread; ++c) t += hp[(size_t)i * kSpread * kSpreadStride + c * kSpreadStride];
            active = (t >> 32) != 0;
        }
        if (!active) break;
        if ((int64_t)r > maxn + 2) return set_error(GBGPU_E_HIP, "batched BFS did not terminate");
        K = std::min(K * 2, 512);
    }
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
// (ms_query_bytes(n) device bytes, ms_pin_bytes() pinned bytes).
int run_ms_group_mem(const std::vector<MsQuery>& qs, void* mem, void* pin, const gbgpu_opts& o,
                     hipStream_t stream, int* rounds) {
    std::vector<std::vector<int>> groups(1);
    for (int i = 0; i < (int)qs.size(); ++i) groups[0].push_back(i);
    int launches = 0;
    *rounds = 0;
    return ms_run_chunk(qs, groups, 0, 1, mem, pin, o, stream, rounds, &launches);
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
