// Compressed adjacency lists and a BFS that reads only them.
//
// The paper keeps its largest inputs in a compressed CSR (the parallel-byte
// code of its "Compression" section: each list cut into blocks that decode
// independently, with per-block offsets, differences within a block).  The
// form here keeps that block structure and swaps the variable-length
// bytes for a layout 64-wide wavefronts decode without a serial pass:
//   * a list is cut into blocks of 64 neighbours;
//   * a block holds its first neighbour (base), a width w = the bit length
//     of (last - base), and then each neighbour's offset from the base,
//     w bits each, packed into 32-bit words (frame of reference);
//   * a list of more than one block starts with a table of the blocks'
//     word offsets from the start of the list.
// Any lane decodes any neighbour with a table read, a header read and one
// bit extract, so push expands compressed lists edge by edge exactly as it
// expands plain ones, and the list order is kept: the first frontier
// neighbour a pull scan meets is still the smallest id.
//
// The BFS follows the paper's BFS algorithm box with the rounds of the
// decomposition code: per round one launch folds the last round's claims
// into the visited bitmap, and one launch pushes (edge-balanced, min-ID
// parent by atomic minimum) or pulls (first frontier neighbour in list
// order), chosen on the device from the frontier's vertex and degree
// totals.  The same kernels also run over the plain lists (gbgpu_bfs_simple)
// so the two list forms are compared with everything else equal.

#include <cstring>

#include <rocprim/device/device_scan.hpp>

#include "common.h"
#include "emit.h"

namespace gb {

constexpr uint32_t kCBlock = 64;  // neighbours per block

struct CAdj {
    uint32_t* words = nullptr;  // the compressed lists
    int64_t* coff = nullptr;    // word offset of each list, n + 1 entries
    int64_t nwords = 0;
    // BFS workspace (sized for n)
    uint32_t* vis = nullptr;
    uint32_t* F[2] = {nullptr, nullptr};
    uint32_t* Q[2] = {nullptr, nullptr};
    uint32_t* P[2] = {nullptr, nullptr};
    unsigned long long* ctl = nullptr;  // qcnt[2], qover[2], max dist, reached; totals at +128
    void* block = nullptr;
};

static void free_lists(CAdj* c) {
    if (c->words) (void)hipFree(c->words);
    if (c->coff) (void)hipFree(c->coff);
    c->words = nullptr;
    c->coff = nullptr;
    c->nwords = 0;
}

void free_cadj(CAdj* c) {
    if (!c) return;
    free_lists(c);
    if (c->block) (void)hipFree(c->block);
    delete c;
}

static int gridv(int64_t items) {
    return (int)std::max<int64_t>(1, std::min<int64_t>((items + kBlock - 1) / kBlock, 4096));
}

__device__ __forceinline__ uint32_t bit_width(uint32_t r) { return r ? 32u - (uint32_t)__clz(r) : 0u; }

// Words of every list: table (lists of more than one block) + per block
// two header words and ceil(len * w / 32) packed words.  vw[n] = 0.
__global__ __launch_bounds__(kBlock) void cz_size_kernel(const int64_t* off, const int32_t* nbr,
                                                         const uint32_t* deg, int64_t n,
                                                         uint32_t* vw) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v <= n; v += stride) {
        if (v == n) {
            vw[n] = 0u;
            continue;
        }
        const uint32_t d = deg[v];
        const uint32_t nb = (d + kCBlock - 1) / kCBlock;
        uint32_t words = nb > 1 ? nb : 0u;
        for (uint32_t k = 0; k < nb; ++k) {
            const int64_t s = off[v] + (int64_t)k * kCBlock;
            const uint32_t len = min(kCBlock, d - k * kCBlock);
            const uint32_t w = bit_width((uint32_t)nbr[s + len - 1] - (uint32_t)nbr[s]);
            words += 2u + (len * w + 31u) / 32u;
        }
        vw[v] = words;
    }
}

// Writes every list: one wavefront per vertex.  The blocks' sizes are
// prefix-summed 64 at a time (lane = block) for the table; then each block
// is written by the whole wavefront: lane e holds offset e, and lane i
// builds packed word i from the (at most 33) offsets that overlap it.
__global__ __launch_bounds__(kBlock) void cz_fill_kernel(const int64_t* off, const int32_t* nbr,
                                                         const uint32_t* deg, int64_t n,
                                                         const int64_t* coff, uint32_t* words) {
    const int l = lane_id();
    const int64_t gw = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t nw = (int64_t)gridDim.x * blockDim.x / kWave;
    for (int64_t v = gw; v < n; v += nw) {
        const uint32_t d = deg[v];
        if (d == 0) continue;  // wave-uniform
        const uint32_t nb = (d + kCBlock - 1) / kCBlock;
        const int64_t vb = coff[v];
        const int64_t s0 = off[v];
        uint32_t run = nb > 1 ? nb : 0u;
        for (uint32_t kb = 0; kb < nb; kb += kWave) {
            const uint32_t k = kb + (uint32_t)l;
            uint32_t size = 0;
            if (k < nb) {
                const int64_t s = s0 + (int64_t)k * kCBlock;
                const uint32_t len = min(kCBlock, d - k * kCBlock);
                const uint32_t w = bit_width((uint32_t)nbr[s + len - 1] - (uint32_t)nbr[s]);
                size = 2u + (len * w + 31u) / 32u;
            }
            const uint32_t incl = wave_incl_sum(size);
            const uint32_t rel = run + incl - size;
            if (k < nb && nb > 1) words[vb + k] = rel;
            run += __shfl(incl, kWave - 1, 64);
            const uint32_t groups = min((uint32_t)kWave, nb - kb);
            for (uint32_t t = 0; t < groups; ++t) {
                const uint32_t kk = kb + t;
                const uint32_t relk = __shfl(rel, (int)t, 64);
                const int64_t s = s0 + (int64_t)kk * kCBlock;
                const uint32_t len = min(kCBlock, d - kk * kCBlock);
                const uint32_t x = (uint32_t)l < len ? (uint32_t)nbr[s + l] : 0u;
                const uint32_t base = __shfl(x, 0, 64);
                const uint32_t last = __shfl(x, (int)len - 1, 64);
                const uint32_t w = bit_width(last - base);
                const uint32_t o = (uint32_t)l < len ? x - base : 0u;
                const int64_t bw = vb + relk;
                if (l == 0) {
                    words[bw] = base;
                    words[bw + 1] = w;
                }
                const uint32_t W = (len * w + 31u) / 32u;
                const uint32_t i = (uint32_t)l;
                const uint32_t e0 = w ? (32u * i) / w : 0u;
                uint32_t acc = 0;
                for (uint32_t q = 0; q < 34u; ++q) {  // uniform: every lane shuffles
                    const uint32_t e = e0 + q;
                    const uint32_t y = __shfl(o, (int)min(e, (uint32_t)kWave - 1u), 64);
                    if (i < W && e < len && (uint64_t)e * w < 32ull * (i + 1)) {
                        const int64_t sh = (int64_t)e * w - 32ll * i;
                        acc |= sh >= 0 ? (uint32_t)((uint64_t)y << sh) : (y >> (uint32_t)(-sh));
                    }
                }
                if (i < W) words[bw + 2 + i] = acc;
            }
        }
    }
}

// Neighbour j of the list starting at word vb (degree d).
__device__ __forceinline__ uint32_t cz_get(const uint32_t* __restrict__ C, int64_t vb, uint32_t d,
                                           uint32_t j) {
    const int64_t bw = vb + (d > kCBlock ? C[vb + (j / kCBlock)] : 0u);
    const uint32_t base = C[bw];
    const uint32_t w = C[bw + 1];
    if (w == 0) return base;
    const uint32_t p = (j % kCBlock) * w;
    const uint32_t* D = C + bw + 2;
    const uint32_t q = p >> 5, r = p & 31u;
    uint64_t x = D[q];
    if (r + w > 32u) x |= (uint64_t)D[q + 1] << 32;
    return base + (uint32_t)((x >> r) & ((1ull << w) - 1ull));
}

__global__ __launch_bounds__(kBlock) void cz_decode_kernel(const uint32_t* words,
                                                           const int64_t* coff,
                                                           const uint32_t* deg,
                                                           const int64_t* off, int64_t n,
                                                           int32_t* out) {
    const int l = lane_id();
    const int64_t gw = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t nw = (int64_t)gridDim.x * blockDim.x / kWave;
    for (int64_t v = gw; v < n; v += nw) {
        const uint32_t d = deg[v];
        const int64_t vb = coff[v];
        for (uint32_t j = (uint32_t)l; j < d; j += kWave)
            out[off[v] + j] = (int32_t)cz_get(words, vb, d, j);
    }
}

// ---------------------------------------------------------------------------
// BFS rounds over either list form
// ---------------------------------------------------------------------------

template <bool kComp>
struct Lists {
    const int64_t* vbase;  // plain: CSR offsets; compressed: word offsets
    const int32_t* nbr;
    const uint32_t* words;
    __device__ __forceinline__ uint32_t get(int64_t vb, uint32_t d, uint32_t j) const {
        if (kComp) return cz_get(words, vb, d, j);
        return (uint32_t)nbr[vb + j];
    }
};

template <bool kComp>
struct CbfsArgs {
    Lists<kComp> L;
    const uint32_t* deg;
    int32_t* dist;
    int32_t* parent;  // INT32_MAX until claimed (the smallest claimer wins)
    uint32_t* vis;
    uint32_t* Fc;
    uint32_t* Fn;
    uint32_t* Qc;
    uint32_t* Pc;
    uint32_t* Qn;
    uint32_t* Pn;
    unsigned long long* qcnt_c;
    unsigned long long* qcnt_n;
    unsigned long long* qover_c;
    unsigned long long* qover_n;
    unsigned long long* tot;
    uint32_t n;
    uint32_t nwords;
    uint64_t dense_at;
    uint32_t light;
};

__global__ __launch_bounds__(kBlock) void cbfs_init_kernel(int64_t n, int64_t nwords, int32_t* dist,
                                                           int32_t* parent, uint32_t* vis,
                                                           uint32_t* F0, uint32_t* F1) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        dist[v] = INT32_MAX;
        parent[v] = INT32_MAX;
    }
    for (int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w < nwords; w += stride) {
        vis[w] = 0u;
        F0[w] = 0u;
        F1[w] = 0u;
    }
}

__global__ void cbfs_seed_kernel(uint32_t src, const uint32_t* deg, int32_t* dist, int32_t* parent,
                                 uint32_t* F0, uint32_t* Q0, uint32_t* P0,
                                 unsigned long long* ctl) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        dist[src] = 0;
        parent[src] = (int32_t)src;
        F0[src >> 5] |= 1u << (src & 31);
        Q0[0] = src;
        P0[0] = 0u;
        ctl[0] = (1ull << 32) | deg[src];
    }
}

// Round r, part 1: last round's claims become visited; the next claim
// bitmap and queue counters are cleared.
template <bool kComp>
__global__ __launch_bounds__(kBlock) void cbfs_fold_kernel(CbfsArgs<kComp> a) {
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t stride = gridDim.x * blockDim.x;
    if (tid == 0) {
        *a.qcnt_n = 0ull;
        *a.qover_n = 0ull;
    }
    for (uint32_t w = tid; w < a.nwords; w += stride) {
        const uint32_t f = a.Fc[w];
        if (f) a.vis[w] |= f;
        a.Fn[w] = 0u;
    }
}

template <bool kComp>
struct CbfsPush {
    const CbfsArgs<kComp>* a;
    WgQueue* q;
    const QueueOut* out;
    uint32_t r1;  // distance of the vertices claimed this round
    static constexpr bool kSkipDead = false;

    __device__ __forceinline__ uint32_t aux(uint32_t u) const { return kComp ? a->deg[u] : 1u; }

    __device__ __forceinline__ void edge(bool act, uint32_t u, uint32_t du, int64_t e, bool) {
        bool take = false;
        uint32_t d = 0, dd = 0;
        if (act) {
            if (kComp) {
                const int64_t vb = a->L.vbase[u];
                d = cz_get(a->L.words, vb, du, (uint32_t)(e - vb));
            } else {
                d = (uint32_t)a->L.nbr[e];
            }
            if (!test_bit(a->vis, d) && (int32_t)u < a->parent[d]) {
                const int32_t old = atomicMin(&a->parent[d], (int32_t)u);
                if (old == INT32_MAX) {
                    take = true;
                    a->dist[d] = (int32_t)r1;
                    dd = a->deg[d];
                    atomicOr(&a->Fn[d >> 5], 1u << (d & 31));
                }
            }
        }
        wgq_push(*q, take, d, dd, *out);
    }

    __device__ __forceinline__ void window_done() {}
};

// Round r, part 2: push over the frontier queue, or pull: every unvisited
// vertex scans its list in order for the first frontier member (a lane
// scans `light` neighbours, then its wavefront the rest, 64 at a time).
template <bool kComp>
__global__ __launch_bounds__(kRBlock, 8) void cbfs_round_kernel(CbfsArgs<kComp> a, uint32_t r,
                                                                uint32_t chunk_cap) {
    __shared__ WgQueue q;
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
    const int l = lane_id();
    if (count == 0) {
        // nothing to expand (the search has ended)
    } else if ((uint64_t)count + edges > a.dense_at) {
        for (uint32_t base = blockIdx.x * (uint32_t)kRBlock; base < a.n;
             base += gridDim.x * (uint32_t)kRBlock) {
            const uint32_t v = base + threadIdx.x;
            const bool unvis = v < a.n && !test_bit(a.vis, v);
            bool take = false;
            uint32_t u = 0, d = 0, j = 0;
            int64_t vb = 0;
            if (unvis) {
                d = a.deg[v];
                vb = a.L.vbase[v];
                const uint32_t lim = min(d, a.light);
                for (; j < lim; ++j) {
                    const uint32_t x = a.L.get(vb, d, j);
                    if (test_bit(a.Fc, x)) {
                        u = x;
                        take = true;
                        break;
                    }
                }
            }
            uint64_t heavy = ballot(unvis && !take && j < d);
            while (heavy) {
                const int h = first_lane(heavy);
                heavy &= heavy - 1ull;
                const uint32_t hj = __shfl(j, h, 64);
                const uint32_t hd = __shfl(d, h, 64);
                const int64_t hvb = (int64_t)shfl64((uint64_t)vb, h);
                uint32_t found = kNone;
                for (uint32_t x0 = hj; x0 < hd; x0 += kWave) {
                    const uint32_t x = x0 + (uint32_t)l;
                    uint32_t y = 0;
                    bool hit = false;
                    if (x < hd) {
                        y = a.L.get(hvb, hd, x);
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
            if (take) {
                a.parent[v] = (int32_t)u;
                a.dist[v] = (int32_t)(r + 1);
            }
            const uint64_t tm = ballot(take);
            if (l == 0 && (uint32_t)tm) a.Fn[v >> 5] = (uint32_t)tm;
            if (l == 32 && (uint32_t)(tm >> 32)) a.Fn[v >> 5] = (uint32_t)(tm >> 32);
            wgq_push(q, take, v, take ? d : 0u, out);
            wgq_maybe_flush(q, out, true, (uint32_t)kRBlock);
        }
    } else if (edges) {
        CbfsPush<kComp> pol{&a, &q, &out, r + 1};
        const uint32_t gwave = blockIdx.x * kRWaves + threadIdx.x / kWave;
        const uint32_t nwaves = gridDim.x * kRWaves;
        const uint32_t wc = wave_chunk(edges, nwaves, chunk_cap);
        const uint32_t nchunks = (edges + wc - 1) / wc;
        for (uint32_t c = gwave; c < nchunks; c += nwaves) {
            const uint32_t eb = c * wc;
            expand_range(a.Qc, a.Pc, count, edges, a.L.vbase, eb, min(edges, eb + wc), pol);
        }
    }
    wgq_finish(q, out, true);
}

// Unclaimed parents back to -1; largest distance and number reached.
__global__ __launch_bounds__(kBlock) void cbfs_final_kernel(int64_t n, const int32_t* dist,
                                                            int32_t* parent,
                                                            unsigned long long* ctl) {
    __shared__ uint32_t smax[kBlock / kWave], scnt[kBlock / kWave];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    uint32_t mx = 0, c = 0;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        const int32_t dv = dist[v];
        if (dv == INT32_MAX) {
            parent[v] = -1;
        } else {
            mx = max(mx, (uint32_t)dv);
            ++c;
        }
    }
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) mx = max(mx, (uint32_t)__shfl_xor(mx, s, 64));
    c = wave_sum(c);
    if (lane_id() == 0) {
        smax[threadIdx.x / kWave] = mx;
        scnt[threadIdx.x / kWave] = c;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t M = 0, C = 0;
        for (int i = 0; i < kBlock / kWave; ++i) {
            M = max(M, smax[i]);
            C += scnt[i];
        }
        atomicMax(&ctl[4], (unsigned long long)M);
        if (C) atomicAdd(&ctl[5], (unsigned long long)C);
    }
}

static int ensure_bfs_ws(gbgpu_graph g, CAdj* c) {
    if (c->block) return GBGPU_OK;
    const int64_t n = g->n;
    const size_t bw = ((size_t)g->nwords * 4 + 255) & ~(size_t)255;
    const size_t qn = ((size_t)(n + 64) * 4 + 255) & ~(size_t)255;
    const size_t total = 3 * bw + 4 * qn + (128 + kSpread * kSpreadStride) * 8;
    if (hipMalloc(&c->block, total) != hipSuccess) {
        c->block = nullptr;
        return set_error(GBGPU_E_NOMEM, "compressed-BFS workspace of %zu bytes", total);
    }
    char* p = (char*)c->block;
    c->vis = (uint32_t*)p; p += bw;
    for (int i = 0; i < 2; ++i) { c->F[i] = (uint32_t*)p; p += bw; }
    for (int i = 0; i < 2; ++i) { c->Q[i] = (uint32_t*)p; p += qn; }
    for (int i = 0; i < 2; ++i) { c->P[i] = (uint32_t*)p; p += qn; }
    c->ctl = (unsigned long long*)p;
    return GBGPU_OK;
}

template <bool kComp>
static int run_cbfs(gbgpu_graph g, int32_t src, int32_t* dist, int32_t* parent,
                    const gbgpu_opts& o, gbgpu_stats* st, hipStream_t s) {
    const double t0 = now_ms();
    CAdj* c = g->cadj;
    GB_TRY(ensure_bfs_ws(g, c));
    const int64_t n = g->n;
    GB_HIP(hipMemsetAsync(c->ctl, 0, 128 * 8, s));
    hipLaunchKernelGGL(cbfs_init_kernel, dim3(gridv(n)), dim3(kBlock), 0, s, n, g->nwords, dist,
                       parent, c->vis, c->F[0], c->F[1]);
    hipLaunchKernelGGL(cbfs_seed_kernel, dim3(1), dim3(64), 0, s, (uint32_t)src, g->deg, dist,
                       parent, c->F[0], c->Q[0], c->P[0], c->ctl);
    GB_HIP(hipGetLastError());
    CbfsArgs<kComp> a;
    a.L.vbase = kComp ? c->coff : g->off;
    a.L.nbr = g->nbr;
    a.L.words = c->words;
    a.deg = g->deg;
    a.dist = dist;
    a.parent = parent;
    a.vis = c->vis;
    a.tot = c->ctl + 128;
    a.n = (uint32_t)n;
    a.nwords = (uint32_t)g->nwords;
    a.dense_at = o.force_direction == 1   ? ~0ull
                 : o.force_direction == 2 ? 0ull
                                          : (uint64_t)(g->m / std::max(1, o.tau));
    a.light = (uint32_t)o.pull_light;
    const int fgrid = gridv(g->nwords);
    const int64_t work = std::max<int64_t>(1, std::max<int64_t>(n / kRBlock, g->m / 4096));
    const int rgrid = (int)std::min<int64_t>(work, o.grid);
    // rounds are queued four at a time; a round after the last one finds an
    // empty frontier and does nothing
    const int ahead = 4;
    uint32_t r = 0;
    for (;;) {
        for (int k = 0; k < ahead; ++k, ++r) {
            a.Fc = c->F[r & 1];
            a.Fn = c->F[(r + 1) & 1];
            a.Qc = c->Q[r & 1];
            a.Pc = c->P[r & 1];
            a.Qn = c->Q[(r + 1) & 1];
            a.Pn = c->P[(r + 1) & 1];
            a.qcnt_c = c->ctl + (r & 1);
            a.qcnt_n = c->ctl + ((r + 1) & 1);
            a.qover_c = c->ctl + 2 + (r & 1);
            a.qover_n = c->ctl + 2 + ((r + 1) & 1);
            hipLaunchKernelGGL(cbfs_fold_kernel<kComp>, dim3(fgrid), dim3(kBlock), 0, s, a);
            hipLaunchKernelGGL(cbfs_round_kernel<kComp>, dim3(rgrid), dim3(kRBlock), 0, s, a, r,
                               (uint32_t)o.wave_chunk);
        }
        GB_HIP(hipGetLastError());
        unsigned long long next = 0;
        GB_HIP(hipMemcpyAsync(&next, c->ctl + (r & 1), 8, hipMemcpyDeviceToHost, s));
        GB_HIP(hipStreamSynchronize(s));
        if ((next >> 32) == 0) break;
        if ((int64_t)r > n + ahead) return set_error(GBGPU_E_HIP, "BFS rounds did not end");
    }
    hipLaunchKernelGGL(cbfs_final_kernel, dim3(std::min(gridv(n), 1024)), dim3(kBlock), 0, s, n,
                       dist, parent, c->ctl);
    GB_HIP(hipGetLastError());
    unsigned long long h[2] = {0, 0};
    GB_HIP(hipMemcpyAsync(h, c->ctl + 4, 16, hipMemcpyDeviceToHost, s));
    GB_HIP(hipStreamSynchronize(s));
    if (st) {
        memset(st, 0, sizeof(*st));
        st->rounds = (int32_t)h[0] + 1;
        st->reached = (int64_t)h[1];
        st->wall_ms = now_ms() - t0;
    }
    return GBGPU_OK;
}

}  // namespace gb

using namespace gb;

extern "C" {

int gbgpu_compress(gbgpu_graph g, int64_t* bytes, void* stream) {
    if (!g) return set_error(GBGPU_E_INVALID, "graph is NULL");
    hipStream_t s = (hipStream_t)stream;
    std::lock_guard<std::mutex> lk(g->mu);
    if (!g->cadj) g->cadj = new CAdj();
    CAdj* c = g->cadj;
    free_lists(c);
    const int64_t n = g->n;
    uint32_t* vw = nullptr;
    void* tmp = nullptr;
    auto fail = [&](int e) {
        if (vw) (void)hipFree(vw);
        if (tmp) (void)hipFree(tmp);
        free_lists(c);
        return e;
    };
    if (hipMalloc(&vw, (size_t)(n + 1) * 4) != hipSuccess ||
        hipMalloc(&c->coff, (size_t)(n + 1) * 8) != hipSuccess)
        return fail(set_error(GBGPU_E_NOMEM, "compression offsets"));
    hipLaunchKernelGGL(cz_size_kernel, dim3(gridv(n + 1)), dim3(kBlock), 0, s, g->off, g->nbr,
                       g->deg, n, vw);
    size_t tb = 0;
    if (rocprim::exclusive_scan(nullptr, tb, vw, c->coff, (int64_t)0, (size_t)n + 1,
                                rocprim::plus<int64_t>(), s) != hipSuccess ||
        hipMalloc(&tmp, std::max<size_t>(tb, 256)) != hipSuccess)
        return fail(set_error(GBGPU_E_NOMEM, "compression scan"));
    if (rocprim::exclusive_scan(tmp, tb, vw, c->coff, (int64_t)0, (size_t)n + 1,
                                rocprim::plus<int64_t>(), s) != hipSuccess)
        return fail(set_error(GBGPU_E_HIP, "compression scan failed"));
    int64_t total = 0;
    if (hipMemcpyAsync(&total, c->coff + n, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(set_error(GBGPU_E_HIP, "compression size read failed"));
    c->nwords = total;
    if (hipMalloc(&c->words, (size_t)std::max<int64_t>(total, 1) * 4 + 8) != hipSuccess)
        return fail(set_error(GBGPU_E_NOMEM, "compressed lists of %lld words", (long long)total));
    const int64_t waves = std::max<int64_t>(1, std::min<int64_t>(n, 65536));
    hipLaunchKernelGGL(cz_fill_kernel, dim3((int)((waves * kWave + kBlock - 1) / kBlock)),
                       dim3(kBlock), 0, s, g->off, g->nbr, g->deg, n, c->coff, c->words);
    const hipError_t e1 = hipGetLastError();
    const hipError_t e2 = hipStreamSynchronize(s);
    (void)hipFree(vw);
    (void)hipFree(tmp);
    vw = nullptr;
    tmp = nullptr;
    if (e1 != hipSuccess || e2 != hipSuccess)
        return fail(set_error(GBGPU_E_HIP, "compression: %s",
                              hipGetErrorString(e1 != hipSuccess ? e1 : e2)));
    if (bytes) *bytes = total * 4 + (n + 1) * 8;
    return GBGPU_OK;
}

int gbgpu_decompress(gbgpu_graph g, int32_t* neighbors, void* stream) {
    if (!g) return set_error(GBGPU_E_INVALID, "graph is NULL");
    if (!neighbors && g->m > 0) return set_error(GBGPU_E_INVALID, "output is NULL");
    std::lock_guard<std::mutex> lk(g->mu);
    if (!g->cadj || !g->cadj->words)
        return set_error(GBGPU_E_INVALID, "graph has no compressed lists (call gbgpu_compress)");
    hipStream_t s = (hipStream_t)stream;
    const int64_t waves = std::max<int64_t>(1, std::min<int64_t>(g->n, 65536));
    hipLaunchKernelGGL(cz_decode_kernel, dim3((int)((waves * kWave + kBlock - 1) / kBlock)),
                       dim3(kBlock), 0, s, g->cadj->words, g->cadj->coff, g->deg, g->off, g->n,
                       neighbors);
    GB_HIP(hipGetLastError());
    GB_HIP(hipStreamSynchronize(s));
    return GBGPU_OK;
}

static int bfs_lists(gbgpu_graph g, int32_t src, int32_t* dist, int32_t* parent,
                     const gbgpu_opts* o, gbgpu_stats* st, void* stream, bool comp) {
    if (!g) return set_error(GBGPU_E_INVALID, "graph is NULL");
    if (!dist || !parent) return set_error(GBGPU_E_INVALID, "output is NULL");
    if (src < 0 || src >= g->n) return set_error(GBGPU_E_INVALID, "src %d out of range", src);
    const gbgpu_opts opt = resolve_opts(o);
    std::lock_guard<std::mutex> lk(g->mu);
    if (comp && (!g->cadj || !g->cadj->words))
        return set_error(GBGPU_E_INVALID, "graph has no compressed lists (call gbgpu_compress)");
    if (!g->cadj) g->cadj = new CAdj();
    hipStream_t s = (hipStream_t)stream;
    const int rc = comp ? run_cbfs<true>(g, src, dist, parent, opt, st, s)
                        : run_cbfs<false>(g, src, dist, parent, opt, st, s);
    // an early error may leave rounds queued that use the workspace
    if (rc != GBGPU_OK) (void)hipStreamSynchronize(s);
    return rc;
}

int gbgpu_bfs_compressed(gbgpu_graph g, int32_t src, int32_t* dist, int32_t* parent,
                         const gbgpu_opts* o, gbgpu_stats* st, void* stream) {
    return bfs_lists(g, src, dist, parent, o, st, stream, true);
}

int gbgpu_bfs_simple(gbgpu_graph g, int32_t src, int32_t* dist, int32_t* parent,
                     const gbgpu_opts* o, gbgpu_stats* st, void* stream) {
    return bfs_lists(g, src, dist, parent, o, st, stream, false);
}

}  // extern "C"
