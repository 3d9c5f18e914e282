// Single-source betweenness centrality.
//
// Method (paper: Betweenness Centrality algorithm box, after Brandes):
//   a forward pass of BFS rounds counts shortest paths -- every vertex of
//   level l adds up the path counts of its neighbours on level l-1 (the
//   box's PathUpdate fetch-and-add) -- and keeps the levels; a backward pass
//   walks the levels from the deepest up, and every vertex u of level l
//   accumulates the dependencies of its neighbours w on level l+1 (the box's
//   DependencyUpdate): delta(u) = sum_w sigma(u) / sigma(w) * (1 + delta(w)).
//   S[v] = delta(v); S[src] = 0 and S = 0 for unreachable vertices.
// Here:
//   * the levels come from the BFS rounds (distances), then a counting sort
//     groups the reached vertices by level and a scan of their degrees in
//     that order gives every level's edges as one contiguous index range;
//   * each level is one launch that walks its vertices' edges in
//     edge-balanced 64-edge windows (as the sparse BFS rounds do); the lanes
//     of one vertex are reduced in registers and the sum is added with one
//     fp64 atomic per vertex and window;
//   * the backward pass keeps acc(u) = sum_w (1 + delta(w)) / sigma(w) =
//     sum_w (1 / sigma(w) + acc(w)), so that delta(u) = sigma(u) * acc(u)
//     needs no division pass per level; S = sigma * acc at the end.
// Path counts and dependencies are fp64 (counts grow exponentially with
// depth); sums are taken in an order the atomics decide, so results match
// a sequential evaluation to rounding, not bit for bit.

#include <cstring>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>
#include <rocprim/iterator/counting_iterator.hpp>

#include "common.h"
#include "emit.h"

namespace gb {

int run_bfs(gbgpu_graph g, int32_t src, int32_t* dist, int32_t* parent, const gbgpu_opts& o,
            gbgpu_stats* st, hipStream_t stream);

struct BcWs {
    int32_t* dist = nullptr;     // BFS levels
    int32_t* par = nullptr;      // BFS parents (unused here)
    uint32_t* cnt = nullptr;     // first position of every level in order (+ the end)
    uint32_t* order = nullptr;   // reached vertices grouped by level
    uint32_t* degO = nullptr;    // their degrees (+ a trailing 0)
    uint32_t* P = nullptr;       // exclusive prefix of degO
    uint32_t* Pb = nullptr;      // sorted level keys, then P at every level boundary
    uint32_t* res = nullptr;     // level mod 3 of every vertex, 2 bits (3 = unreached)
    double* sigma = nullptr;
    double* acc = nullptr;
    void* scan_tmp = nullptr;
    size_t scan_bytes = 0;
    void* block = nullptr;
    hipEvent_t done = nullptr;
};

void free_bc_ws(BcWs* w) {
    if (!w) return;
    if (w->done) {
        (void)hipEventSynchronize(w->done);
        (void)hipEventDestroy(w->done);
    }
    if (w->scan_tmp) (void)hipFree(w->scan_tmp);
    if (w->block) (void)hipFree(w->block);
    delete w;
}

static size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

static int ensure_bc_ws(gbgpu_graph g) {
    if (g->bc) return GBGPU_OK;
    const int64_t n = g->n;
    const size_t u32n = a256((size_t)(n + 64) * 4), f64n = a256((size_t)n * 8);
    const size_t resn = a256((size_t)(n / 16 + 64) * 4);
    const size_t total = 2 * u32n + 5 * u32n + resn + 2 * f64n;
    BcWs* w = new BcWs();
    hipError_t e = hipMalloc(&w->block, total);
    if (e != hipSuccess) {
        delete w;
        return set_error(GBGPU_E_NOMEM, "betweenness workspace of %zu bytes: %s", total,
                         hipGetErrorString(e));
    }
    char* p = (char*)w->block;
    w->dist = (int32_t*)p; p += u32n;
    w->par = (int32_t*)p; p += u32n;
    w->cnt = (uint32_t*)p; p += u32n;
    w->order = (uint32_t*)p; p += u32n;
    w->degO = (uint32_t*)p; p += u32n;
    w->P = (uint32_t*)p; p += u32n;
    w->Pb = (uint32_t*)p; p += u32n;
    w->res = (uint32_t*)p; p += resn;
    w->sigma = (double*)p; p += f64n;
    w->acc = (double*)p;
    size_t tb = 0, ts = 0;
    if (rocprim::exclusive_scan(nullptr, tb, w->degO, w->P, 0u, (size_t)(n + 1),
                                rocprim::plus<uint32_t>()) != hipSuccess ||
        rocprim::radix_sort_pairs(nullptr, ts, (const uint32_t*)w->dist, w->Pb,
                                  rocprim::counting_iterator<uint32_t>(0u), w->order,
                                  (unsigned int)n, 0u, 32u) != hipSuccess ||
        hipMalloc(&w->scan_tmp, std::max<size_t>(std::max(tb, ts), 256)) != hipSuccess ||
        hipEventCreateWithFlags(&w->done, hipEventDisableTiming) != hipSuccess) {
        free_bc_ws(w);
        return set_error(GBGPU_E_NOMEM, "betweenness scan / sort workspace");
    }
    w->scan_bytes = std::max<size_t>(std::max(tb, ts), 256);
    g->bc = w;
    return GBGPU_OK;
}

__global__ __launch_bounds__(kBlock) void bc_depth_kernel(const int32_t* dist, int64_t n,
                                                          uint32_t* depth) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int32_t mx = -1;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride)
        if (dist[v] != INT32_MAX) mx = max(mx, dist[v]);
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) mx = max(mx, __shfl_xor(mx, d, 64));
    if (lane_id() == 0 && mx >= 0) atomicMax(depth, (uint32_t)mx + 1u);
}

// Level boundaries in the level-sorted keys: base[l] = first position of
// level l (levels are contiguous: every level below the depth is
// non-empty); base[levels] = number of reached vertices (unreached keys,
// INT32_MAX, sort last).
__global__ __launch_bounds__(kBlock) void bc_boundary_kernel(const uint32_t* key, int64_t n,
                                                             uint32_t levels, uint32_t* base) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint32_t k = min(key[i], levels);
        const uint32_t kp = i == 0 ? 0xFFFFFFFFu : min(key[i - 1], levels);
        if (k != kp) base[k] = (uint32_t)i;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && min(key[n - 1], levels) < levels)
        base[levels] = (uint32_t)n;
}

__global__ __launch_bounds__(kBlock) void bc_degree_kernel(const uint32_t* order, uint32_t R,
                                                           const uint32_t* deg, uint32_t* degO) {
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i <= R; i += stride)
        degO[i] = i < R ? deg[order[i]] : 0u;
}

__global__ void bc_bounds_kernel(const uint32_t* P, const uint32_t* base, int32_t levels,
                                 uint32_t* Pb) {
    const int32_t i = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i <= levels) Pb[i] = P[base[i]];
}

// Neighbours' levels differ by at most one, so level mod 3 tells a vertex's
// parents (level - 1), peers and children (level + 1) apart.  Packed 16
// vertices to a word, the residues take n / 4 bytes: the per-edge test reads
// them instead of the 4-byte distances, and they fit in the L2.
__global__ __launch_bounds__(kBlock) void bc_residue_kernel(const int32_t* dist, int64_t n,
                                                            uint32_t* res) {
    const int64_t words = (n + 15) / 16;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t wd = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; wd < words; wd += stride) {
        uint32_t x = 0u;
        for (int i = 0; i < 16; ++i) {
            const int64_t v = wd * 16 + i;
            uint32_t r = 3u;
            if (v < n && dist[v] != INT32_MAX) r = (uint32_t)dist[v] % 3u;
            x |= r << (2 * i);
        }
        res[wd] = x;
    }
}

__device__ __forceinline__ uint32_t level_res(const uint32_t* res, uint32_t u) {
    return (res[u >> 4] >> ((u & 15u) * 2u)) & 3u;
}

__global__ __launch_bounds__(kBlock) void bc_init_kernel(double* sigma, double* acc, int64_t n,
                                                         int32_t src) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        sigma[v] = v == src ? 1.0 : 0.0;
        acc[v] = 0.0;
    }
}

__global__ __launch_bounds__(kBlock) void bc_output_kernel(const double* sigma, const double* acc,
                                                           const int32_t* dist, int64_t n,
                                                           int32_t src, double* dep) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride)
        dep[v] = (v != src && dist[v] != INT32_MAX) ? sigma[v] * acc[v] : 0.0;
}

struct BcArgs {
    const int64_t* off;
    const int32_t* nbr;
    const uint32_t* res;  // level mod 3, packed
    const uint32_t* Q;   // this level's vertices
    const uint32_t* P;   // their absolute degree prefix
    uint32_t cnt;
    uint32_t e0, e1;     // this level's absolute edge range
    uint32_t want;       // residue of the neighbours this pass reads
    uint32_t chunk;
    double* sigma;
    double* acc;
};

__device__ __forceinline__ double shfl_down_f64(double x, int d) {
    const unsigned long long b = __double_as_longlong(x);
    const uint32_t lo = __shfl_down((uint32_t)b, d, 64);
    const uint32_t hi = __shfl_down((uint32_t)(b >> 32), d, 64);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Per edge (v, u) of a level-l vertex v: forward, sigma(u) when u is on
// level l-1; backward, 1 / sigma(u) + acc(u) when u is on level l+1 (told
// apart by the level residues).  The
// lanes of one v are contiguous in a window; their sum goes to v with one
// atomic.
template <bool kForward>
struct BcPolicy {
    const BcArgs* a;
    static constexpr bool kSkipDead = false;

    __device__ __forceinline__ uint32_t aux(uint32_t) const { return 1u; }

    __device__ __forceinline__ void edge(bool act, uint32_t v, uint32_t, int64_t e, bool) {
        const int l = lane_id();
        double c = 0.0;
        const uint32_t owner = act ? v : 0xFFFFFFFFu;
        if (act) {
            const uint32_t u = (uint32_t)a->nbr[e];
            if (level_res(a->res, u) == a->want)
                c = kForward ? a->sigma[u] : 1.0 / a->sigma[u] + a->acc[u];
        }
#pragma unroll
        for (int dd = 1; dd < 64; dd <<= 1) {
            const double oc = shfl_down_f64(c, dd);
            const uint32_t oo = __shfl_down(owner, dd, 64);
            if (l + dd < 64 && oo == owner) c += oc;
        }
        const uint32_t prev = __shfl_up(owner, 1, 64);
        if (act && (l == 0 || prev != owner) && c != 0.0)
            atomicAdd(kForward ? &a->sigma[v] : &a->acc[v], c);
    }

    __device__ __forceinline__ void window_done() {}
};

template <bool kForward>
__global__ __launch_bounds__(kRBlock, 8) void bc_level_kernel(BcArgs a) {
    const uint32_t gwave = blockIdx.x * kRWaves + threadIdx.x / kWave;
    const uint32_t nwaves = gridDim.x * kRWaves;
    const uint32_t E = a.e1 - a.e0;
    const uint32_t nchunks = (E + a.chunk - 1) / a.chunk;
    BcPolicy<kForward> pol{&a};
    for (uint32_t c = gwave; c < nchunks; c += nwaves) {
        const uint32_t eb = a.e0 + c * a.chunk;
        expand_range(a.Q, a.P, a.cnt, a.e1, a.off, eb, min(a.e1, eb + a.chunk), pol);
    }
}

static int grid_n(int64_t items) {
    return (int)std::max<int64_t>(1, std::min<int64_t>((items + kBlock - 1) / kBlock, 4096));
}

}  // namespace gb

using namespace gb;

extern "C" {

int gbgpu_bc(gbgpu_graph g, int32_t src, double* dep, const gbgpu_opts* o, gbgpu_stats* st,
             void* stream) {
    if (!g) return set_error(GBGPU_E_INVALID, "graph is NULL");
    if (!dep) return set_error(GBGPU_E_INVALID, "output is NULL");
    if (src < 0 || src >= g->n)
        return set_error(GBGPU_E_INVALID, "src %d out of range [0, %lld)", src, (long long)g->n);
    const double t0 = now_ms();
    const gbgpu_opts opt = resolve_opts(o);
    hipStream_t s = (hipStream_t)stream;
    std::lock_guard<std::mutex> lk(g->mu);
    GB_TRY(ensure_bc_ws(g));
    BcWs* w = g->bc;
    GB_HIP(hipStreamWaitEvent(s, w->done, 0));
    // 1. levels: the BFS rounds (depth = largest finite distance + 1)
    GB_TRY(run_bfs(g, src, w->dist, w->par, opt, nullptr, s));
    GB_HIP(hipMemsetAsync(w->Pb, 0, 4, s));
    hipLaunchKernelGGL(bc_depth_kernel, dim3(grid_n(g->n)), dim3(kBlock), 0, s, w->dist, g->n,
                       w->Pb);
    GB_HIP(hipGetLastError());
    uint32_t depth = 0;
    GB_HIP(hipMemcpyAsync(&depth, w->Pb, 4, hipMemcpyDeviceToHost, s));
    GB_HIP(hipStreamSynchronize(s));
    const int32_t levels = (int32_t)std::max<uint32_t>(depth, 1u);
    // 2. reached vertices grouped by level (radix sort of (level, id) over
    //    the bits the depth needs; INT32_MAX of unreached vertices has them
    //    all set and sorts last), then their degrees in that order
    unsigned int bits = 1;
    while ((1u << bits) <= (uint32_t)levels) ++bits;
    size_t tb = w->scan_bytes;
    GB_HIP(rocprim::radix_sort_pairs(w->scan_tmp, tb, (const uint32_t*)w->dist, w->Pb,
                                     rocprim::counting_iterator<uint32_t>(0u), w->order,
                                     (unsigned int)g->n, 0u, bits, s));
    hipLaunchKernelGGL(bc_boundary_kernel, dim3(grid_n(g->n)), dim3(kBlock), 0, s, w->Pb, g->n,
                       (uint32_t)levels, w->cnt);
    GB_HIP(hipGetLastError());
    std::vector<uint32_t> base((size_t)levels + 1), cnt((size_t)levels);
    GB_HIP(hipMemcpyAsync(base.data(), w->cnt, ((size_t)levels + 1) * 4, hipMemcpyDeviceToHost,
                          s));
    GB_HIP(hipStreamSynchronize(s));
    for (int32_t l = 0; l < levels; ++l) cnt[(size_t)l] = base[(size_t)l + 1] - base[(size_t)l];
    const uint32_t R = base[(size_t)levels];
    hipLaunchKernelGGL(bc_degree_kernel, dim3(grid_n((int64_t)R + 1)), dim3(kBlock), 0, s,
                       w->order, R, g->deg, w->degO);
    GB_HIP(hipGetLastError());
    tb = w->scan_bytes;
    GB_HIP(rocprim::exclusive_scan(w->scan_tmp, tb, w->degO, w->P, 0u, (size_t)R + 1,
                                   rocprim::plus<uint32_t>(), s));
    // 3. every level's edge range: P at the level boundaries
    hipLaunchKernelGGL(bc_bounds_kernel, dim3((levels + 1 + 255) / 256), dim3(256), 0, s, w->P,
                       w->cnt, levels, w->Pb);
    std::vector<uint32_t> pb((size_t)levels + 1);
    GB_HIP(hipMemcpyAsync(pb.data(), w->Pb, ((size_t)levels + 1) * 4, hipMemcpyDeviceToHost, s));
    hipLaunchKernelGGL(bc_residue_kernel, dim3(grid_n((g->n + 15) / 16)), dim3(kBlock), 0, s,
                       w->dist, g->n, w->res);
    hipLaunchKernelGGL(bc_init_kernel, dim3(grid_n(g->n)), dim3(kBlock), 0, s, w->sigma, w->acc,
                       g->n, src);
    GB_HIP(hipGetLastError());
    GB_HIP(hipStreamSynchronize(s));
    // 4. forward (levels 1 .. L-1), then backward (levels L-2 .. 1)
    BcArgs a;
    a.off = g->off;
    a.nbr = g->nbr;
    a.res = w->res;
    a.sigma = w->sigma;
    a.acc = w->acc;
    int64_t launches = 0;
    auto level_launch = [&](int32_t l, bool fwd) -> int {
        a.Q = w->order + base[(size_t)l];
        a.P = w->P + base[(size_t)l];
        a.cnt = cnt[(size_t)l];
        a.e0 = pb[(size_t)l];
        a.e1 = pb[(size_t)l + 1];
        a.want = (uint32_t)((fwd ? l + 2 : l + 1) % 3);  // (l - 1) mod 3 / (l + 1) mod 3
        if (a.cnt == 0 || a.e1 == a.e0) return GBGPU_OK;
        const uint32_t E = a.e1 - a.e0;
        const uint32_t nw = (uint32_t)opt.grid * kRWaves;
        uint32_t c = (E + nw - 1) / nw;
        c = std::max<uint32_t>(64u, std::min<uint32_t>((uint32_t)opt.wave_chunk, (c + 63u) & ~63u));
        a.chunk = c;
        const uint32_t chunks = (E + c - 1) / c;
        const int grid = (int)std::max<uint32_t>(1, std::min<uint32_t>((chunks + kRWaves - 1) / kRWaves,
                                                                      (uint32_t)opt.grid));
        if (fwd)
            hipLaunchKernelGGL(bc_level_kernel<true>, dim3(grid), dim3(kRBlock), 0, s, a);
        else
            hipLaunchKernelGGL(bc_level_kernel<false>, dim3(grid), dim3(kRBlock), 0, s, a);
        ++launches;
        return hipGetLastError() == hipSuccess ? GBGPU_OK
                                               : set_error(GBGPU_E_HIP, "level kernel launch failed");
    };
    for (int32_t l = 1; l < levels; ++l) GB_TRY(level_launch(l, true));
    for (int32_t l = levels - 2; l >= 1; --l) GB_TRY(level_launch(l, false));
    hipLaunchKernelGGL(bc_output_kernel, dim3(grid_n(g->n)), dim3(kBlock), 0, s, w->sigma, w->acc,
                       w->dist, g->n, src, dep);
    GB_HIP(hipGetLastError());
    GB_HIP(hipEventRecord(w->done, s));
    GB_HIP(hipStreamSynchronize(s));
    if (st) {
        memset(st, 0, sizeof(*st));
        st->rounds = levels;
        st->reached = R;
        st->launches = (int32_t)launches;
        st->wall_ms = now_ms() - t0;
    }
    return GBGPU_OK;
}

}  // extern "C"
