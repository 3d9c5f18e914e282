// Query server: resident graphs, per-query workspaces carved from a
// caller-provided device arena, admission by footprint, continuous batching.
//
// Workers (one HIP stream each, default priority) take work from a FIFO of
// pending queries.  A worker that becomes free takes the oldest query; for a
// BFS on a graph known to be shallow and of at most 2^24 vertices it also
// takes every other pending BFS on the same graph (up to 64) and runs them
// together as one bit-packed multi-source traversal.  Work is
// admitted only when its device footprint fits in the arena's free space, so
// the server never allocates device memory of its own; queries that arrive
// while others run are picked up as soon as a worker and memory are free, and
// run concurrently with them on the device.  A weighted query whose distance
// buckets outgrow their capacity is re-queued at the front with twice the
// capacity (its outputs are then rewritten from scratch).

#include <condition_variable>
#include <deque>
#include <map>
#include <thread>
#include <unordered_map>
#include <unordered_set>

#include "common.h"
#include "admission.h"

namespace gb {

size_t bfs_ws_bytes(int64_t n, int64_t nwords);
void bfs_ws_attach(BfsWs* w, void* mem, int64_t n, int64_t nwords);
int bfs_ws_host_init(BfsWs* w);
BfsWs* bfs_ws_new();
int run_bfs_ws(gbgpu_graph g, BfsWs* w, int32_t src, int32_t* dist, int32_t* parent,
               const gbgpu_opts& o, gbgpu_stats* st, hipStream_t stream, bool sync_end,
               bool wait_prev);
uint32_t wbfs_window(int32_t maxw, int32_t req);
uint32_t wbfs_default_capacity(int64_t n);
size_t wbfs_bytes(int64_t n, uint32_t NB, uint32_t C);
void wbfs_ws_attach(WbfsWs* w, void* mem, int64_t n, uint32_t NB, uint32_t C);
int wbfs_ws_host_init(WbfsWs* w);
WbfsWs* wbfs_ws_new();
int run_wbfs_ws(gbgpu_graph g, WbfsWs* w, int32_t src, uint32_t* dist, int32_t* parent,
                const gbgpu_opts& o, gbgpu_stats* st, hipStream_t stream, bool* overflow);
size_t ms_query_bytes(int64_t n, int64_t k);
size_t ms_pin_bytes();
int run_ms_group_mem(const std::vector<MsQuery>& qs, void* mem, void* pin, const gbgpu_opts& o,
                     hipStream_t stream, int* rounds, uint32_t kcap, const MsJoinHook* hook);

// Bucket capacity of a weighted query: the re-queue override, else the
// option, else the default.
static uint32_t initial_capacity(gbgpu_graph g, uint32_t cap_override, const gbgpu_opts& o) {
    if (cap_override) return cap_override;
    if (o.bucket_capacity > 0) return (uint32_t)std::min<int64_t>(o.bucket_capacity, g->n);
    return wbfs_default_capacity(g->n);
}

size_t query_footprint(gbgpu_graph g, int kind, uint32_t cap_override, const gbgpu_opts& o) {
    if (kind == GBGPU_QUERY_BFS) return bfs_ws_bytes(g->n, g->nwords);
    const uint32_t NB = wbfs_window(g->maxw, o.bucket_window);
    return wbfs_bytes(g->n, NB, initial_capacity(g, cap_override, o));
}

struct Worker {
    hipStream_t stream = nullptr;
    BfsWs* bws = nullptr;
    WbfsWs* wws = nullptr;
    void* pin = nullptr;
    std::thread th;
};

}  // namespace gb

struct gbgpu_server_s {
    char* arena = nullptr;
    size_t arena_bytes = 0;
    gb::ArenaAlloc alloc{0};
    int device = 0;
    gbgpu_opts opts;
    std::vector<gbgpu_graph> graphs;
    std::vector<uint32_t> wcap;       // per graph: bucket capacity a weighted query needed
    std::vector<gb::CapWindow> capwin;  // per graph: bucket fills since wcap last changed
    gb::SchedEnv env;                 // admission rule's view of the graphs
    std::mutex mu;
    std::condition_variable cv;       // work available / memory freed / stop
    std::condition_variable cv_idle;  // everything finished
    std::deque<gb::PendingQ> pending;
    size_t max_pending = 1 << 16;
    std::unordered_map<uint64_t, gbgpu_result> done;
    std::unordered_set<uint64_t> live;
    uint64_t next_ticket = 1;
    int running = 0;
    bool stop = false;
    std::vector<gb::Worker*> workers;
};

namespace gb {

static void finish_query(gbgpu_server sv, const PendingQ& p, int status, int rounds, int64_t t_start,
                         int32_t batch, int32_t launches) {
    gbgpu_result r;
    memset(&r, 0, sizeof(r));
    r.status = status;
    r.rounds = rounds - p.join_round;
    r.t_arrive_ns = p.t_arrive;
    r.t_start_ns = p.t_start ? p.t_start : t_start;
    r.t_done_ns = now_ns();
    r.retries = p.retries;
    r.batch = batch;
    r.join_round = p.join_round;
    r.launches = launches;
    sv->done[p.ticket] = r;
    sv->live.erase(p.ticket);
}

static void worker_loop(gbgpu_server sv, Worker* w) {
    (void)hipSetDevice(sv->device);
    std::unique_lock<std::mutex> lk(sv->mu);
    for (;;) {
        // take the oldest query whose footprint fits now (with the other
        // pending BFS queries on its graph when they can be bit-packed)
        std::vector<PendingQ> job;
        size_t off = 0, bytes = 0;
        uint32_t kcap = 0;
        while (!sv->stop) {
            if (sched_admit(sv->pending, sv->alloc, sv->env, sv->wcap, &job, &off, &bytes, &kcap))
                break;
            sv->cv.wait(lk);
        }
        if (job.empty()) break;  // stopping
        ++sv->running;
        lk.unlock();
        const int64_t t_start = now_ns();
        void* mem = sv->arena + off;
        gbgpu_graph g = sv->graphs[job[0].q.graph_id];
        int status = GBGPU_OK, rounds = 0, launches = 0;
        uint32_t peak = 0;  // weighted query without overflow: its fullest bucket
        bool requeue = false;
        uint32_t usedcap = 0;
        if (job.size() > 1) {
            std::vector<MsQuery> qs;
            for (auto& p : job) qs.push_back(MsQuery{g, p.q.src, (int32_t*)p.q.dist, p.q.parent});
            // BFS queries on this graph that arrive while the group runs join
            // it at a round boundary, while it has free source slots
            const int32_t gid = job[0].q.graph_id;
            MsJoinHook hook = [&](uint32_t r, int room, bool, std::vector<MsQuery>* add) {
                std::lock_guard<std::mutex> lk2(sv->mu);
                if (sv->stop) return;
                std::vector<PendingQ> got;
                sched_take_bfs(sv->pending, gid, room, &got);
                const int64_t t = now_ns();
                for (auto& p : got) {
                    p.t_start = t;
                    p.join_round = (int32_t)r;
                    add->push_back(MsQuery{g, p.q.src, (int32_t*)p.q.dist, p.q.parent});
                    job.push_back(p);
                }
            };
            status = run_ms_group_mem(qs, mem, w->pin, sv->opts, w->stream, &rounds, kcap,
                                      kcap > job.size() ? &hook : nullptr);
        } else if (job[0].q.kind == GBGPU_QUERY_BFS) {
            bfs_ws_attach(w->bws, mem, g->n, g->nwords);
            gbgpu_stats st{};
            status = run_bfs_ws(g, w->bws, job[0].q.src, (int32_t*)job[0].q.dist, job[0].q.parent,
                                sv->opts, &st, w->stream, true, true);  // the arena is reused at once
            rounds = st.rounds;
            launches = st.launches;
        } else {
            const uint32_t NB = wbfs_window(g->maxw, sv->opts.bucket_window);
            const uint32_t C = initial_capacity(g, job[0].cap, sv->opts);
            wbfs_ws_attach(w->wws, mem, g->n, NB, C);
            gbgpu_stats st{};
            bool overflow = false;
            status = run_wbfs_ws(g, w->wws, job[0].q.src, (uint32_t*)job[0].q.dist, job[0].q.parent,
                                 sv->opts, &st, w->stream, &overflow);
            rounds = st.rounds;
            launches = st.launches;
            if (status == GBGPU_OK && overflow) {
                requeue = true;
                usedcap = C;
            } else if (status == GBGPU_OK) {
                peak = (uint32_t)std::max(st.bucket_peak, 0);
            }
        }
        lk.lock();
        sv->alloc.release(off, bytes);
        --sv->running;
        if (peak) {
            const int32_t gid = job[0].q.graph_id;
            sched_note_peak(sv->wcap[gid], sv->capwin[gid], peak, initial_capacity(g, 0, sv->opts));
        }
        if (requeue) {
            // re-queued at the front with twice the buckets; failed when the
            // larger workspace could never be admitted
            if (!sched_requeue_overflow(sv->pending, sv->env, sv->wcap, sv->arena_bytes, job[0],
                                        usedcap, g->n))
                finish_query(sv, job[0], GBGPU_E_NOMEM, rounds, t_start, 1, launches);
        } else {
            for (auto& p : job)
                finish_query(sv, p, status, rounds, t_start, (int32_t)job.size(), launches);
        }
        sv->cv.notify_all();
        if (sv->pending.empty() && sv->running == 0) sv->cv_idle.notify_all();
    }
}

}  // namespace gb

using namespace gb;

extern "C" {

int gbgpu_debug_arena_selftest(uint64_t seed, int32_t steps) {
    // randomized check of the first-fit arena against a reference bitmap
    const size_t units = 512;
    ArenaAlloc a(units * 256);
    std::vector<char> used(units, 0);
    std::vector<std::pair<size_t, size_t>> live;
    uint64_t x = seed * 0x9E3779B97F4A7C15ull + 1;
    auto rnd = [&]() { x ^= x << 13; x ^= x >> 7; x ^= x << 17; return x; };
    for (int i = 0; i < steps; ++i) {
        if (live.empty() || rnd() % 3) {
            const size_t bytes = 1 + rnd() % (40 * 256);
            size_t off = 0;
            const size_t need = (bytes + 255) / 256;
            bool fit_exists = false;
            for (size_t s0 = 0; s0 + need <= units && !fit_exists; ++s0) {
                bool ok = true;
                for (size_t k = 0; k < need && ok; ++k) ok = !used[s0 + k];
                fit_exists = ok;
            }
            const bool got = a.alloc(bytes, &off);
            if (got != fit_exists) return set_error(GBGPU_E_INVALID, "fit mismatch at step %d", i);
            if (got) {
                if (off % 256 || off / 256 + need > units) return set_error(GBGPU_E_INVALID, "bad offset");
                for (size_t k = 0; k < need; ++k) {
                    if (used[off / 256 + k]) return set_error(GBGPU_E_INVALID, "overlap at step %d", i);
                    used[off / 256 + k] = 1;
                }
                live.emplace_back(off, bytes);
            }
        } else {
            const size_t j = rnd() % live.size();
            a.release(live[j].first, live[j].second);
            const size_t need = (live[j].second + 255) / 256;
            for (size_t k = 0; k < need; ++k) used[live[j].first / 256 + k] = 0;
            live.erase(live.begin() + j);
        }
    }
    for (auto& l : live) a.release(l.first, l.second);
    if (a.largest() != units * 256) return set_error(GBGPU_E_INVALID, "free ranges did not coalesce");
    return GBGPU_OK;
}

int gbgpu_query_footprint(gbgpu_graph g, int32_t kind, size_t* bytes) {
    if (!g || !bytes) return set_error(GBGPU_E_INVALID, "bad argument");
    if (kind != GBGPU_QUERY_BFS && kind != GBGPU_QUERY_WBFS)
        return set_error(GBGPU_E_INVALID, "unknown query kind %d", kind);
    gbgpu_opts o = resolve_opts(nullptr);
    *bytes = query_footprint(g, kind, 0, o);
    return GBGPU_OK;
}

int gbgpu_server_create(void* arena, size_t arena_bytes, int32_t max_inflight, const gbgpu_opts* o,
                        gbgpu_server* out) {
    if (!out) return set_error(GBGPU_E_INVALID, "out is NULL");
    if (!arena || arena_bytes == 0) return set_error(GBGPU_E_INVALID, "empty arena");
    if (max_inflight < 1 || max_inflight > 64)
        return set_error(GBGPU_E_INVALID, "max_inflight must be in [1, 64]");
    gbgpu_server sv = new gbgpu_server_s();
    sv->arena = (char*)arena;
    sv->arena_bytes = arena_bytes;
    sv->alloc = ArenaAlloc(arena_bytes & ~(size_t)255);
    sv->opts = resolve_opts(o);
    if (sv->opts.max_pending > 0) sv->max_pending = (size_t)sv->opts.max_pending;
    // BFS queries are bit-packed only on graphs a single-source search has
    // shown to be shallow, and only up to 2^24 vertices; the others run one
    // at a time (concurrently on the workers).  A packed group holds every
    // query in it until its last round, hundreds of rounds on a deep graph;
    // on RMAT scale 26, 64 bit-packed sources ran at 312 queries/s against
    // 358 one at a time (measured with the earlier two-array staging).  The
    // graph list is only read under the server's lock.
    sv->env.packable = [sv](int32_t gid) {
        gbgpu_graph g = sv->graphs[gid];
        const int32_t depth = g->depth.load(std::memory_order_relaxed);
        return depth > 0 && depth <= kDeepGraph && g->n <= kPackedMaxN;
    };
    sv->env.footprint = [sv](int32_t gid, int32_t kind, uint32_t cap) {
        return query_footprint(sv->graphs[gid], kind, cap, sv->opts);
    };
    sv->env.packed_bytes = [sv](int32_t gid, int64_t k) {
        return ms_query_bytes(sv->graphs[gid]->n, k);
    };
    if (hipGetDevice(&sv->device) != hipSuccess) {
        delete sv;
        return set_error(GBGPU_E_HIP, "hipGetDevice failed");
    }
    for (int i = 0; i < max_inflight; ++i) {
        Worker* w = new Worker();
        w->bws = bfs_ws_new();
        w->wws = wbfs_ws_new();
        int st = GBGPU_OK;
        if (hipStreamCreateWithFlags(&w->stream, hipStreamNonBlocking) != hipSuccess)
            st = set_error(GBGPU_E_HIP, "stream creation failed");
        if (st == GBGPU_OK) st = bfs_ws_host_init(w->bws);
        if (st == GBGPU_OK) st = wbfs_ws_host_init(w->wws);
        if (st == GBGPU_OK && hipHostMalloc(&w->pin, ms_pin_bytes(), hipHostMallocDefault) != hipSuccess)
            st = set_error(GBGPU_E_HIP, "pinned buffer allocation failed");
        if (st != GBGPU_OK) {
            free_bfs_ws(w->bws);
            free_wbfs_ws(w->wws);
            if (w->pin) (void)hipHostFree(w->pin);
            if (w->stream) (void)hipStreamDestroy(w->stream);
            delete w;
            gbgpu_server_destroy(sv);
            return st;
        }
        sv->workers.push_back(w);
    }
    for (Worker* w : sv->workers) w->th = std::thread(worker_loop, sv, w);
    *out = sv;
    return GBGPU_OK;
}

int gbgpu_server_add_graph(gbgpu_server sv, gbgpu_graph g, int32_t* graph_id) {
    if (!sv || !g || !graph_id) return set_error(GBGPU_E_INVALID, "bad argument");
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->graphs.push_back(g);
    sv->wcap.push_back(0u);
    sv->capwin.push_back(CapWindow{});
    *graph_id = (int32_t)sv->graphs.size() - 1;
    return GBGPU_OK;
}

int gbgpu_submit(gbgpu_server sv, const gbgpu_query* q, uint64_t* ticket) {
    if (!sv || !q || !ticket) return set_error(GBGPU_E_INVALID, "bad argument");
    const int64_t t = now_ns();
    std::lock_guard<std::mutex> lk(sv->mu);
    if (q->graph_id < 0 || q->graph_id >= (int32_t)sv->graphs.size())
        return set_error(GBGPU_E_INVALID, "unknown graph id %d", q->graph_id);
    gbgpu_graph g = sv->graphs[q->graph_id];
    if (q->kind != GBGPU_QUERY_BFS && q->kind != GBGPU_QUERY_WBFS)
        return set_error(GBGPU_E_INVALID, "unknown query kind %d", q->kind);
    if (q->src < 0 || q->src >= g->n) return set_error(GBGPU_E_INVALID, "source out of range");
    if (!q->dist || !q->parent) return set_error(GBGPU_E_INVALID, "NULL output");
    if (q->kind == GBGPU_QUERY_WBFS) {
        if (!g->w) return set_error(GBGPU_E_INVALID, "graph has no weights");
        if (g->minw < 1) return set_error(GBGPU_E_INVALID, "weighted BFS needs weights >= 1");
        if (g->maxw > 2047) return set_error(GBGPU_E_UNSUPPORTED, "max weight exceeds 2047");
        if ((uint64_t)std::max(g->maxw, 1) * (uint64_t)g->n >= 0xFFFFFFFEull)
            return set_error(GBGPU_E_OVERFLOW, "max_weight * n must stay below 2^32 - 2");
    }
    if (query_footprint(g, q->kind, 0, sv->opts) > sv->arena_bytes)
        return set_error(GBGPU_E_NOMEM, "query footprint exceeds the arena");
    if (sv->stop) return set_error(GBGPU_E_INVALID, "server is stopping");
    if (sv->pending.size() >= sv->max_pending) return set_error(GBGPU_E_AGAIN, "pending queue full");
    PendingQ p;
    p.ticket = sv->next_ticket++;
    p.q = *q;
    p.t_arrive = t;
    p.cap = 0;
    p.retries = 0;
    p.t_start = 0;
    p.join_round = 0;
    sv->pending.push_back(p);
    sv->live.insert(p.ticket);
    *ticket = p.ticket;
    sv->cv.notify_one();
    return GBGPU_OK;
}

int gbgpu_poll(gbgpu_server sv, uint64_t ticket, gbgpu_result* r) {
    if (!sv || !r) return set_error(GBGPU_E_INVALID, "bad argument");
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->done.find(ticket);
    if (it != sv->done.end()) {
        *r = it->second;
        sv->done.erase(it);
        return GBGPU_OK;
    }
    if (sv->live.count(ticket)) return set_error(GBGPU_E_AGAIN, "query %llu not finished",
                                                 (unsigned long long)ticket);
    return set_error(GBGPU_E_NOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
}

int gbgpu_server_drain(gbgpu_server sv) {
    if (!sv) return set_error(GBGPU_E_INVALID, "server is NULL");
    std::unique_lock<std::mutex> lk(sv->mu);
    sv->cv_idle.wait(lk, [&] { return sv->pending.empty() && sv->running == 0; });
    return GBGPU_OK;
}

int gbgpu_server_destroy(gbgpu_server sv) {
    if (!sv) return set_error(GBGPU_E_INVALID, "server is NULL");
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
        sv->cv.notify_all();
    }
    for (Worker* w : sv->workers) {
        if (w->th.joinable()) w->th.join();
        free_bfs_ws(w->bws);
        free_wbfs_ws(w->wws);
        if (w->pin) (void)hipHostFree(w->pin);
        if (w->stream) (void)hipStreamDestroy(w->stream);
        delete w;
    }
    delete sv;
    return GBGPU_OK;
}

}  // extern "C"
