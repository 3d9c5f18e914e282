// Graph handles, load-time validation, options, errors, and the C entry
// points for single-source traversal.
//
// The CSR layout (Preliminaries, "Graph Notation": vertices 0..n-1, no self
// edges or duplicates; CSR/CSC formats) is used as given: int64 offsets,
// int32 neighbours sorted ascending, optional int32 weights aligned with the
// neighbours.  Graphs are symmetric, so a vertex's list serves as both its
// out-edges (sparse push) and in-edges (dense pull).

#include <time.h>

#include <thread>

#include "common.h"

namespace gb {

static thread_local std::string t_last_error;

int set_error(int status, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    t_last_error = buf;
    return status;
}

double now_ms() {
    timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return ts.tv_sec * 1e3 + ts.tv_nsec * 1e-6;
}

int64_t now_ns() {
    timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (int64_t)ts.tv_sec * 1000000000ll + ts.tv_nsec;
}

int host_log_alloc(HostLog* hl, size_t log_steps) {
    const size_t bytes = (kHostLogOff + 4 * log_steps) * 4;
    if (hipHostMalloc((void**)&hl->h, bytes, hipHostMallocMapped | hipHostMallocCoherent) !=
        hipSuccess) {
        hl->h = nullptr;
        return set_error(GBGPU_E_NOMEM, "pinned progress/log buffer of %zu bytes", bytes);
    }
    memset(hl->h, 0, bytes);
    if (hipHostGetDevicePointer((void**)&hl->d, hl->h, 0) != hipSuccess) {
        host_log_free(hl);
        return set_error(GBGPU_E_HIP, "no device address for the pinned progress buffer");
    }
    return GBGPU_OK;
}

void host_log_free(HostLog* hl) {
    if (hl->h) (void)hipHostFree(hl->h);
    hl->h = hl->d = nullptr;
}

static inline void cpu_relax() { __builtin_ia32_pause(); }

int run_pipeline(volatile uint32_t* prog, hipStream_t stream, int ahead, int64_t max_launches,
                 const std::function<void(int64_t)>& launch, int64_t* issued_out) {
    ahead = std::max(ahead, 1);
    int64_t issued = 0;
    auto top_up = [&](int64_t upto) {
        upto = std::min(upto, max_launches);
        for (; issued < upto; ++issued) launch(issued);
    };
    top_up(ahead);
    GB_HIP(hipGetLastError());
    // Every launch that finds work writes prog[0] when it starts and the
    // first one that finds none writes prog[1], so the progress words alone
    // keep the queue topped up.  The stream itself is queried only after
    // kQuietMs without a new progress word (a failed device, or launches
    // exhausted): the runtime answers a query on a busy stream by queueing
    // a marker, which costs every launch behind it a few microseconds.
    constexpr double kQuietMs = 2.0;
    int64_t seen = -1;
    double quiet_since = 0.0;
    for (uint64_t spin = 1;; ++spin) {
        if (prog[1]) break;
        const int64_t started = prog[0];
        if (issued < started + ahead && issued < max_launches) {
            top_up(started + ahead);
            GB_HIP(hipGetLastError());
            continue;
        }
        if ((spin & 255u) == 0) {
            const double t = now_ms();
            if (started != seen) {
                seen = started;
                quiet_since = t;
            } else if (t - quiet_since > kQuietMs) {
                quiet_since = t;
                const hipError_t e = hipStreamQuery(stream);
                if (e == hipSuccess) {
                    if (prog[1]) break;
                    if (issued >= max_launches)
                        return set_error(GBGPU_E_HIP,
                                         "traversal did not finish within %lld launches",
                                         (long long)max_launches);
                    top_up(issued + ahead);
                    GB_HIP(hipGetLastError());
                } else if (e != hipErrorNotReady) {
                    return set_error(GBGPU_E_HIP, "traversal stream failed: %s",
                                     hipGetErrorString(e));
                }
            }
        }
        if ((spin & 4095u) == 0) std::this_thread::yield(); else cpu_relax();
    }
    *issued_out = issued;
    return GBGPU_OK;
}

gbgpu_opts resolve_opts(const gbgpu_opts* o) {
    gbgpu_opts r;
    memset(&r, 0, sizeof(r));
    if (o) r = *o;
    if (r.force_direction < 0 || r.force_direction > 3) r.force_direction = 0;
    // reserved[kTauDefaulted] tells the traversals that pick their own
    // threshold (weighted BFS) that the caller left tau unset
    r.reserved[kTauDefaulted] = r.tau <= 0 ? 1 : 0;
    if (r.tau <= 0) r.tau = 20;
    if (r.pull_light <= 0) r.pull_light = 32;
    if (r.wave_chunk <= 0) r.wave_chunk = 256;
    r.wave_chunk = std::max(64, (r.wave_chunk + 63) & ~63);
    if (r.grid <= 0) r.grid = 512;
    if (r.rounds_per_sync <= 0) r.rounds_per_sync = 3;
    if (r.beta == 0) r.beta = 24;
    if (r.bucket_window < 0) r.bucket_window = 0;
    if (r.bucket_capacity < 0) r.bucket_capacity = 0;
    return r;
}

int run_bfs(gbgpu_graph g, int32_t src, int32_t* dist, int32_t* parent, const gbgpu_opts& o,
            gbgpu_stats* st, hipStream_t stream);
int run_bfs_many(gbgpu_graph g, const int32_t* srcs, int32_t k, int32_t* dist, int32_t* parent,
                 int64_t stride, const gbgpu_opts& o, gbgpu_stats* st, hipStream_t stream);
int run_bfs_noalloc(gbgpu_graph g, int32_t src, int32_t* dist, int32_t* parent,
                    const gbgpu_opts& o, gbgpu_stats* st, hipStream_t stream);
int run_wbfs(gbgpu_graph g, int32_t src, uint32_t* dist, int32_t* parent, const gbgpu_opts& o,
             gbgpu_stats* st, hipStream_t stream);
int bfs_round_log(gbgpu_graph g, uint32_t* out, int32_t max_rounds, int32_t* nrounds);
int wbfs_step_log(gbgpu_graph g, uint32_t* out, int32_t max_steps, int32_t* nsteps);

// ---------------------------------------------------------------------------
// load-time kernels
// ---------------------------------------------------------------------------
enum : uint32_t {
    VF_OFFSETS = 1u,
    VF_RANGE = 2u,
    VF_ORDER = 4u,
    VF_SELF = 8u,
    VF_ASYM = 16u,
    VF_WASYM = 64u,
};

__global__ void check_offsets_kernel(const int64_t* off, int64_t n, int64_t m, uint32_t* flag) {
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; v < n; v += stride) {
        int64_t a = off[v], b = off[v + 1];
        if (a > b || a < 0 || b > m) atomicOr(flag, VF_OFFSETS);
        if (v == 0 && a != 0) atomicOr(flag, VF_OFFSETS);
        if (v == n - 1 && b != m) atomicOr(flag, VF_OFFSETS);
    }
}

// Binary search for x in the sorted list of vertex v; returns its edge index
// or -1.
__device__ int64_t find_in_list(const int64_t* off, const int32_t* nbr, int64_t v, int32_t x) {
    int64_t lo = off[v], hi = off[v + 1];
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        int32_t y = nbr[mid];
        if (y == x) return mid;
        if (y < x) lo = mid + 1; else hi = mid;
    }
    return -1;
}

// Weight range: *maxw = largest weight (when >= 1), *below = largest 1 - w
// over weights below 1 (0 when every weight is >= 1).
__device__ __forceinline__ void note_weight_range(int32_t lmax, uint32_t lbelow, int32_t* maxw,
                                                  uint32_t* below) {
    if (lmax > 0) atomicMax(maxw, lmax);
    if (lbelow) atomicMax(below, lbelow);
}

__global__ void check_edges_kernel(const int64_t* off, const int32_t* nbr, const int32_t* w,
                                   int64_t n, uint32_t* flag, int32_t* maxw, uint32_t* below) {
    int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; u < n; u += stride) {
        int32_t prev = -1;
        int32_t lmax = 0;
        uint32_t lbelow = 0;
        for (int64_t e = off[u]; e < off[u + 1]; ++e) {
            int32_t v = nbr[e];
            if (v < 0 || v >= n) { atomicOr(flag, VF_RANGE); continue; }
            if (v <= prev) atomicOr(flag, VF_ORDER);
            prev = v;
            if (v == u) atomicOr(flag, VF_SELF);
            int64_t back = find_in_list(off, nbr, v, (int32_t)u);
            if (back < 0) atomicOr(flag, VF_ASYM);
            if (w) {
                if (back >= 0 && w[back] != w[e]) atomicOr(flag, VF_WASYM);
                lmax = max(lmax, w[e]);
                if (w[e] < 1) lbelow = max(lbelow, (uint32_t)(1 - (int64_t)w[e]));
            }
        }
        if (w) note_weight_range(lmax, lbelow, maxw, below);
    }
}

__global__ void weight_range_kernel(const int32_t* w, int64_t m, int32_t* maxw, uint32_t* below) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int32_t lm = 0;
    uint32_t lb = 0;
    for (; e < m; e += stride) {
        const int32_t x = w[e];
        lm = max(lm, x);
        if (x < 1) lb = max(lb, (uint32_t)(1 - (int64_t)x));
    }
    for (int d = 32; d >= 1; d >>= 1) {
        lm = max(lm, __shfl_xor(lm, d, 64));
        lb = max(lb, (uint32_t)__shfl_xor(lb, d, 64));
    }
    if (lane_id() == 0) note_weight_range(lm, lb, maxw, below);
}

// Degrees, the bitmap of vertices of degree <= 1, and the head of every
// list: its first four
// neighbours (kNone-padded) in one 16-byte record, so a dense scan that stops
// early reads them with one coalesced load instead of one random line of the
// neighbour array per vertex.
__global__ void degree_kernel(const int64_t* off, const int32_t* nbr, int64_t n, int64_t nwords,
                              uint32_t* deg, uint32_t* pruned, uint4* head) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = t; v < n; v += stride) {
        const int64_t s0 = off[v];
        const int64_t d = off[v + 1] - s0;
        deg[v] = (uint32_t)d;
        uint32_t h[4];
        for (int i = 0; i < 4; ++i) h[i] = i < d ? (uint32_t)nbr[s0 + i] : kNone;
        head[v] = make_uint4(h[0], h[1], h[2], h[3]);
    }
    for (int64_t w = t; w < nwords; w += stride) {
        uint32_t bits = 0;
        for (int b = 0; b < 32; ++b) {
            int64_t v = w * 32 + b;
            if (v >= n || off[v + 1] - off[v] <= 1) bits |= 1u << b;
        }
        pruned[w] = bits;
    }
}

static int grid_for(int64_t items) {
    int64_t g = (items + kBlock - 1) / kBlock;
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, 8192));
}

__global__ void gather_head_kernel(const uint4* head, const uint32_t* core, uint32_t ncore,
                                   uint4* core_head) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < ncore; i += gridDim.x * blockDim.x)
        core_head[i] = head[core[i]];
}

// fills in the neighbour half of each (vertex, neighbour) leaf record
__global__ void leaf_nbr_kernel(const int64_t* off, const int32_t* nbr, uint2* leaf,
                                uint32_t nleaf) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nleaf; i += gridDim.x * blockDim.x)
        leaf[i].y = (uint32_t)nbr[off[leaf[i].x]];
}

// Dense-scan plan: work items that cover every non-isolated vertex once.
// An item is either a run of at most 64 consecutive vertices with at most
// kPlanCap edges in total ({first, end, kPlanHub, 0}), or a piece of at most
// kPlanCap edges of one vertex whose list is longer ({v, v + 1, first_edge,
// end_edge}).  Runs of isolated vertices are skipped.
int ensure_pull_plan(gbgpu_graph g) {
    std::lock_guard<std::mutex> lk(g->plan_mu);
    if (g->plan) return GBGPU_OK;
    std::vector<int64_t> off((size_t)g->n + 1);
    GB_HIP(hipMemcpy(off.data(), g->off, off.size() * 8, hipMemcpyDeviceToHost));
    std::vector<uint4> items;
    items.reserve((size_t)(g->m / kPlanCap + g->n / 64 + 16));
    int64_t i = 0;
    const int64_t n = g->n;
    while (i < n) {
        const int64_t d = off[i + 1] - off[i];
        if (d == 0) {
            ++i;
            continue;
        }
        if (d > (int64_t)kPlanCap) {
            for (int64_t e = off[i]; e < off[i + 1]; e += kPlanCap)
                items.push_back(make_uint4((uint32_t)i, (uint32_t)(i + 1), (uint32_t)e,
                                           (uint32_t)std::min<int64_t>(e + kPlanCap, off[i + 1])));
            ++i;
            continue;
        }
        const int64_t vb = i;
        int64_t edges = 0;
        while (i < n && i - vb < 64) {
            const int64_t di = off[i + 1] - off[i];
            if (di > (int64_t)kPlanCap || edges + di > (int64_t)kPlanCap) break;
            edges += di;
            ++i;
        }
        items.push_back(make_uint4((uint32_t)vb, (uint32_t)i, kPlanHub, 0u));
    }
    // vertex lists for the BFS: degree >= 2 (scanned by dense rounds) and
    // degree 1 (attached after the rounds through their one neighbour)
    std::vector<uint32_t> corev;
    std::vector<uint2> leafv;
    corev.reserve((size_t)n);
    int64_t maxd = 0;
    for (int64_t v = 0; v < n; ++v) {
        const int64_t d = off[v + 1] - off[v];
        maxd = std::max(maxd, d);
        if (d >= 2) corev.push_back((uint32_t)v);
        else if (d == 1) leafv.push_back(make_uint2((uint32_t)v, 0u));
    }
    uint32_t* d_core = nullptr;
    uint4* d_core_head = nullptr;
    uint2* d_leaf = nullptr;
    auto free_lists = [&]() {
        if (d_core) (void)hipFree(d_core);
        if (d_core_head) (void)hipFree(d_core_head);
        if (d_leaf) (void)hipFree(d_leaf);
    };
    if (hipMalloc(&d_core, std::max<size_t>(corev.size(), 1) * 4) != hipSuccess ||
        hipMalloc(&d_core_head, std::max<size_t>(corev.size(), 1) * sizeof(uint4)) != hipSuccess ||
        hipMalloc(&d_leaf, std::max<size_t>(leafv.size(), 1) * sizeof(uint2)) != hipSuccess) {
        free_lists();
        return set_error(GBGPU_E_NOMEM, "vertex list allocation failed");
    }
    if ((!corev.empty() &&
         hipMemcpy(d_core, corev.data(), corev.size() * 4, hipMemcpyHostToDevice) != hipSuccess) ||
        (!leafv.empty() && hipMemcpy(d_leaf, leafv.data(), leafv.size() * sizeof(uint2),
                                     hipMemcpyHostToDevice) != hipSuccess)) {
        free_lists();
        return set_error(GBGPU_E_HIP, "vertex list upload failed");
    }
    if (!corev.empty()) {
        hipLaunchKernelGGL(gather_head_kernel, dim3(grid_for((int64_t)corev.size())), dim3(kBlock),
                           0, 0, g->head, d_core, (uint32_t)corev.size(), d_core_head);
        if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
            free_lists();
            return set_error(GBGPU_E_HIP, "head record gather failed");
        }
    }
    if (!leafv.empty()) {
        hipLaunchKernelGGL(leaf_nbr_kernel, dim3(grid_for((int64_t)leafv.size())), dim3(kBlock), 0, 0,
                           g->off, g->nbr, d_leaf, (uint32_t)leafv.size());
        if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
            free_lists();
            return set_error(GBGPU_E_HIP, "leaf neighbour kernel failed");
        }
    }
    uint4* d_items = nullptr;
    if (hipMalloc(&d_items, std::max<size_t>(items.size(), 1) * sizeof(uint4)) != hipSuccess) {
        free_lists();
        return set_error(GBGPU_E_NOMEM, "dense-scan plan allocation failed");
    }
    if (!items.empty() &&
        hipMemcpy(d_items, items.data(), items.size() * sizeof(uint4), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(d_items);
        free_lists();
        return set_error(GBGPU_E_HIP, "dense-scan plan upload failed");
    }
    g->plan = d_items;
    g->nplan = (uint32_t)items.size();
    g->core = d_core;
    g->max_degree = maxd;
    g->core_head = d_core_head;
    g->ncore = (uint32_t)corev.size();
    g->leaf = d_leaf;
    g->nleaf = (uint32_t)leafv.size();
    return GBGPU_OK;
}



}  // namespace gb

using namespace gb;

extern "C" {

const char* gbgpu_last_error(void) { return t_last_error.c_str(); }

int gbgpu_version(void) { return 10000; }

int gbgpu_load_csr(int64_t n, int64_t m, const int64_t* offsets, const int32_t* neighbors,
                   const int32_t* weights, uint32_t flags, void* stream, gbgpu_graph* out) {
    if (!out) return set_error(GBGPU_E_INVALID, "out is NULL");
    if (!offsets) return set_error(GBGPU_E_INVALID, "offsets is NULL");
    if (m > 0 && !neighbors) return set_error(GBGPU_E_INVALID, "neighbors is NULL");
    if (n <= 0) return set_error(GBGPU_E_INVALID, "n must be positive (got %lld)", (long long)n);
    if (m < 0) return set_error(GBGPU_E_INVALID, "m must be non-negative");
    if (n >= (1ll << 31) - 1)
        return set_error(GBGPU_E_UNSUPPORTED, "n = %lld exceeds 2^31 - 2", (long long)n);
    if (m >= (1ll << 31))
        return set_error(GBGPU_E_UNSUPPORTED, "m = %lld: at most 2^31 - 1 stored edges",
                         (long long)m);
    if (!(flags & GBGPU_SYMMETRIC))
        return set_error(GBGPU_E_INVALID,
                         "GBGPU_SYMMETRIC is required: dense rounds read a vertex's own list "
                         "as its in-edges");
    hipStream_t s = (hipStream_t)stream;
    gbgpu_graph g = new gbgpu_graph_s();
    g->n = n;
    g->m = m;
    g->off = offsets;
    g->nbr = neighbors;
    g->w = weights;
    g->nwords = ((n + 63) / 64) * 2;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) { delete g; return set_error(GBGPU_E_HIP, "hipGetDevice failed"); }
    g->device = dev;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
        g->num_cus = cus;
    uint32_t* scratch = nullptr;  // [0] flag, [1] max weight, [2] largest 1 - w below 1
    auto fail = [&](int st) {
        if (g->deg) (void)hipFree(g->deg);
        if (g->pruned) (void)hipFree(g->pruned);
        if (g->head) (void)hipFree(g->head);
        if (scratch) (void)hipFree(scratch);
        delete g;
        return st;
    };
    if (hipMalloc(&g->deg, (size_t)n * 4) != hipSuccess ||
        hipMalloc(&g->pruned, (size_t)g->nwords * 4) != hipSuccess ||
        hipMalloc(&g->head, (size_t)n * sizeof(uint4)) != hipSuccess ||
        hipMalloc(&scratch, 16) != hipSuccess)
        return fail(set_error(GBGPU_E_NOMEM, "graph metadata allocation failed"));
    if (hipMemsetAsync(scratch, 0, 16, s) != hipSuccess)
        return fail(set_error(GBGPU_E_HIP, "hipMemsetAsync failed"));
    uint32_t host[4] = {0, 0, 0, 0};
    if (flags & GBGPU_VALIDATE) {
        hipLaunchKernelGGL(check_offsets_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, offsets, n,
                           m, scratch);
        if (hipMemcpyAsync(host, scratch, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return fail(set_error(GBGPU_E_HIP, "offset validation failed to run"));
        if (host[0]) return fail(set_error(GBGPU_E_INVALID, "invalid offsets (non-monotone, "
                                           "offsets[0] != 0 or offsets[n] != m)"));
        if (m > 0) {
            hipLaunchKernelGGL(check_edges_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, offsets,
                               neighbors, weights, n, scratch, (int32_t*)(scratch + 1),
                               scratch + 2);
            if (hipMemcpyAsync(host, scratch, 12, hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess)
                return fail(set_error(GBGPU_E_HIP, "edge validation failed to run"));
            uint32_t f = host[0];
            if (f & VF_RANGE) return fail(set_error(GBGPU_E_INVALID, "neighbour id out of range"));
            if (f & VF_ORDER)
                return fail(set_error(GBGPU_E_INVALID, "adjacency list not strictly ascending"));
            if (f & VF_SELF) return fail(set_error(GBGPU_E_INVALID, "self loop"));
            if (f & VF_ASYM) return fail(set_error(GBGPU_E_INVALID, "graph is not symmetric"));
            if (f & VF_WASYM) return fail(set_error(GBGPU_E_INVALID, "weights are not symmetric"));
        }
    } else if (weights && m > 0) {
        hipLaunchKernelGGL(weight_range_kernel, dim3(grid_for(m)), dim3(kBlock), 0, s, weights, m,
                           (int32_t*)(scratch + 1), scratch + 2);
        if (hipMemcpyAsync(host, scratch, 12, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return fail(set_error(GBGPU_E_HIP, "weight range kernel failed"));
    }
    g->maxw = weights ? (int32_t)host[1] : 0;
    g->minw = (weights && m > 0 && host[2]) ? (int32_t)(1 - (int64_t)host[2]) : 1;
    if (g->minw < 1 && !(flags & GBGPU_SIGNED_WEIGHTS))
        return fail(set_error(GBGPU_E_INVALID,
                              "weight %d < 1 (load with GBGPU_SIGNED_WEIGHTS for general-weight "
                              "SSSP)", g->minw));
    hipLaunchKernelGGL(degree_kernel, dim3(grid_for(std::max<int64_t>(n, g->nwords))), dim3(kBlock),
                       0, s, offsets, neighbors, n, g->nwords, g->deg, g->pruned, g->head);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
        return fail(set_error(GBGPU_E_HIP, "degree kernel failed"));
    (void)hipFree(scratch);
    scratch = nullptr;
    int ps = ensure_pull_plan(g);
    if (ps != GBGPU_OK) return fail(ps);
    *out = g;
    return GBGPU_OK;
}

int gbgpu_graph_free(gbgpu_graph g) {
    if (!g) return set_error(GBGPU_E_INVALID, "graph is NULL");
    {
        std::lock_guard<std::mutex> lk(g->mu);
        free_bfs_ws(g->bfs);
        free_bfs_ws(g->sr);
        free_bc_ws(g->bc);
        free_arena(g->cc);
        free_cadj(g->cadj);
        free_wbfs_ws(g->wbfs);
        free_multi_ws(g->multi);
        if (g->plan) (void)hipFree(g->plan);
        if (g->core) (void)hipFree(g->core);
        if (g->core_head) (void)hipFree(g->core_head);
        if (g->leaf) (void)hipFree(g->leaf);
        if (g->wsort_nbr) (void)hipFree(g->wsort_nbr);
        if (g->wsort_w) (void)hipFree(g->wsort_w);
        (void)hipFree(g->deg);
        (void)hipFree(g->pruned);
        (void)hipFree(g->head);
    }
    delete g;
    return GBGPU_OK;
}

int gbgpu_graph_info(gbgpu_graph g, int64_t* n, int64_t* m, int32_t* max_weight) {
    if (!g) return set_error(GBGPU_E_INVALID, "graph is NULL");
    if (n) *n = g->n;
    if (m) *m = g->m;
    if (max_weight) *max_weight = g->maxw;
    return GBGPU_OK;
}

int gbgpu_bfs(gbgpu_graph g, int32_t src, int32_t* dist, int32_t* parent, const gbgpu_opts* o,
              gbgpu_stats* st, void* stream) {
    if (!g) return set_error(GBGPU_E_INVALID, "graph is NULL");
    if (!dist || !parent) return set_error(GBGPU_E_INVALID, "dist/parent is NULL");
    if (src < 0 || src >= g->n)
        return set_error(GBGPU_E_INVALID, "src %d out of range [0, %lld)", src, (long long)g->n);
    gbgpu_opts opt = resolve_opts(o);
    std::lock_guard<std::mutex> lk(g->mu);
    return run_bfs(g, src, dist, parent, opt, st, (hipStream_t)stream);
}

int gbgpu_bfs_noalloc(gbgpu_graph g, int32_t src, int32_t* dist, int32_t* parent,
                      const gbgpu_opts* o, gbgpu_stats* st, void* stream) {
    if (!g) return set_error(GBGPU_E_INVALID, "graph is NULL");
    if (!dist || !parent) return set_error(GBGPU_E_INVALID, "dist/parent is NULL");
    if (src < 0 || src >= g->n)
        return set_error(GBGPU_E_INVALID, "src %d out of range [0, %lld)", src, (long long)g->n);
    gbgpu_opts opt = resolve_opts(o);
    return run_bfs_noalloc(g, src, dist, parent, opt, st, (hipStream_t)stream);
}

int gbgpu_bfs_many(gbgpu_graph g, const int32_t* srcs, int32_t k, int32_t* dist,
                   int32_t* parent, int64_t row_stride, const gbgpu_opts* o, gbgpu_stats* st,
                   void* stream) {
    if (!g) return set_error(GBGPU_E_INVALID, "graph is NULL");
    if (!srcs || k < 1) return set_error(GBGPU_E_INVALID, "need k >= 1 sources");
    if (!dist || !parent) return set_error(GBGPU_E_INVALID, "dist/parent is NULL");
    if (row_stride != 0 && row_stride < g->n)
        return set_error(GBGPU_E_INVALID, "row_stride must be 0 or at least n");
    for (int32_t i = 0; i < k; ++i)
        if (srcs[i] < 0 || srcs[i] >= g->n)
            return set_error(GBGPU_E_INVALID, "srcs[%d] = %d out of range [0, %lld)", i, srcs[i],
                             (long long)g->n);
    gbgpu_opts opt = resolve_opts(o);
    std::lock_guard<std::mutex> lk(g->mu);
    return run_bfs_many(g, srcs, k, dist, parent, row_stride, opt, st, (hipStream_t)stream);
}

int gbgpu_wbfs(gbgpu_graph g, int32_t src, uint32_t* dist, int32_t* parent, const gbgpu_opts* o,
               gbgpu_stats* st, void* stream) {
    if (!g) return set_error(GBGPU_E_INVALID, "graph is NULL");
    if (!g->w) return set_error(GBGPU_E_INVALID, "graph was loaded without weights");
    if (g->minw < 1) return set_error(GBGPU_E_INVALID, "weighted BFS needs weights >= 1");
    if (!dist || !parent) return set_error(GBGPU_E_INVALID, "dist/parent is NULL");
    if (src < 0 || src >= g->n)
        return set_error(GBGPU_E_INVALID, "src %d out of range [0, %lld)", src, (long long)g->n);
    if (g->maxw > 2047)
        return set_error(GBGPU_E_UNSUPPORTED, "max weight %d exceeds 2047", g->maxw);
    if ((uint64_t)std::max(g->maxw, 1) * (uint64_t)g->n >= 0xFFFFFFFEull)
        return set_error(GBGPU_E_OVERFLOW, "max_weight * n must stay below 2^32 - 2");
    gbgpu_opts opt = resolve_opts(o);
    std::lock_guard<std::mutex> lk(g->mu);
    return run_wbfs(g, src, dist, parent, opt, st, (hipStream_t)stream);
}

// Diagnostic: per-round log of the last BFS on g (4 words per round).
int gbgpu_debug_bfs_log(gbgpu_graph g, uint32_t* out, int32_t max_rounds, int32_t* nrounds) {
    if (!g || !out || !nrounds) return set_error(GBGPU_E_INVALID, "bad argument");
    std::lock_guard<std::mutex> lk(g->mu);
    return bfs_round_log(g, out, max_rounds, nrounds);
}

// Diagnostic: per-step log of the last wBFS on g (4 words per bucket step).
int gbgpu_debug_wbfs_log(gbgpu_graph g, uint32_t* out, int32_t max_steps, int32_t* nsteps) {
    if (!g || !out || !nsteps) return set_error(GBGPU_E_INVALID, "bad argument");
    std::lock_guard<std::mutex> lk(g->mu);
    return wbfs_step_log(g, out, max_steps, nsteps);
}

}  // extern "C"
