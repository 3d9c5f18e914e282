// CPU unit tests of the query server's scheduling rules (admission.h) with fake
// graphs and footprints; built and run under address and undefined-behaviour
// sanitizers by test_host_sanitized.py.  Prints one line per failed check
// and exits non-zero if any failed.
#include <stdio.h>

#include <deque>
#include <vector>

#include "admission.h"

using namespace gb;

static int failures = 0;
#define CHECK(cond)                                                        \
    do {                                                                   \
        if (!(cond)) {                                                     \
            printf("FAIL %s:%d: %s\n", __FILE__, __LINE__, #cond);         \
            ++failures;                                                    \
        }                                                                  \
    } while (0)

static uint64_t next_ticket = 1;
static PendingQ q(int32_t gid, int32_t kind, int32_t src) {
    PendingQ p{};
    p.ticket = next_ticket++;
    p.q.graph_id = gid;
    p.q.kind = kind;
    p.q.src = src;
    p.t_arrive = (int64_t)p.ticket * 1000;  // fake clock: arrival order
    return p;
}

// Fake environment: graph 0 packable, graph 1 not; a BFS costs 100 units of
// 256 bytes, a weighted query 300 + cap units, k packed BFS 20 + 60 k.
static SchedEnv fake_env(std::vector<bool> packable) {
    SchedEnv e;
    e.packable = [packable](int32_t gid) { return (bool)packable[gid]; };
    e.footprint = [](int32_t, int32_t kind, uint32_t cap) {
        return (size_t)256 * (kind == GBGPU_QUERY_BFS ? 100 : 300 + (cap ? cap : 64));
    };
    e.packed_bytes = [](int32_t, int64_t k) { return (size_t)256 * (20 + 60 * k); };
    return e;
}

static void test_oldest_first_alone() {
    std::deque<PendingQ> pend = {q(1, GBGPU_QUERY_BFS, 5), q(0, GBGPU_QUERY_WBFS, 6)};
    ArenaAlloc a(256 * 10000);
    std::vector<uint32_t> cap = {0, 0};
    std::vector<PendingQ> job;
    size_t off = 0, bytes = 0;
    uint32_t kc = 0;
    CHECK(sched_admit(pend, a, fake_env({true, false}), cap, &job, &off, &bytes, &kc));
    CHECK(job.size() == 1 && job[0].q.src == 5);  // graph 1 is not packable
    CHECK(bytes == 256 * 100 && off == 0 && kc == 0);
    CHECK(pend.size() == 1 && pend.front().q.src == 6);
}

static void test_packs_same_graph_bfs_in_order() {
    std::deque<PendingQ> pend;
    for (int i = 0; i < 5; ++i) pend.push_back(q(0, GBGPU_QUERY_BFS, i));
    pend.push_back(q(0, GBGPU_QUERY_WBFS, 100));
    pend.push_back(q(1, GBGPU_QUERY_BFS, 101));
    for (int i = 5; i < 8; ++i) pend.push_back(q(0, GBGPU_QUERY_BFS, i));
    ArenaAlloc a(256 * 10000);
    std::vector<uint32_t> cap = {0, 0};
    std::vector<PendingQ> job;
    size_t off = 0, bytes = 0;
    uint32_t kc = 0;
    CHECK(sched_admit(pend, a, fake_env({true, false}), cap, &job, &off, &bytes, &kc));
    CHECK(job.size() == 8);
    for (size_t i = 0; i < job.size(); ++i) CHECK(job[i].q.src == (int32_t)i);
    // the workspace fits a group of 64: later arrivals may join it
    CHECK(bytes == 256 * (20 + 60 * 64) && kc == 64);
    // the others keep their order
    CHECK(pend.size() == 2 && pend[0].q.src == 100 && pend[1].q.src == 101);
}

static void test_pack_limit_and_halving() {
    std::deque<PendingQ> pend;
    for (int i = 0; i < 70; ++i) pend.push_back(q(0, GBGPU_QUERY_BFS, i));
    std::vector<uint32_t> cap = {0};
    std::vector<PendingQ> job;
    size_t off = 0, bytes = 0;
    uint32_t kc = 0;
    {
        ArenaAlloc a(256 * 10000);
        std::deque<PendingQ> p = pend;
        CHECK(sched_admit(p, a, fake_env({true}), cap, &job, &off, &bytes, &kc));
        CHECK(job.size() == 64 && p.size() == 6 && p.front().q.src == 64 && kc == 64);
    }
    {
        // room for 600 units: groups of 64, 32 and 16 do not fit, 8 does
        // (and no room for arrivals to join)
        ArenaAlloc a(256 * 600);
        std::deque<PendingQ> p = pend;
        CHECK(sched_admit(p, a, fake_env({true}), cap, &job, &off, &bytes, &kc));
        CHECK(job.size() == 8 && bytes == 256 * 500 && kc == 8);
        CHECK(job.front().q.src == 0 && job.back().q.src == 7);
    }
    {
        // not even two fit (140 units): the oldest runs alone (100 units)
        ArenaAlloc a(256 * 120);
        std::deque<PendingQ> p = pend;
        CHECK(sched_admit(p, a, fake_env({true}), cap, &job, &off, &bytes, &kc));
        CHECK(job.size() == 1 && job[0].q.src == 0 && kc == 0);
    }
}

static void test_take_bfs_for_a_joining_round() {
    // what a running group on graph 0 takes at a round boundary: the first
    // BFS queries on graph 0, in order, up to its free slots; others stay
    std::deque<PendingQ> pend = {q(0, GBGPU_QUERY_WBFS, 1), q(0, GBGPU_QUERY_BFS, 2),
                                 q(1, GBGPU_QUERY_BFS, 3), q(0, GBGPU_QUERY_BFS, 4),
                                 q(0, GBGPU_QUERY_BFS, 5)};
    std::vector<PendingQ> got;
    sched_take_bfs(pend, 0, 2, &got);
    CHECK(got.size() == 2 && got[0].q.src == 2 && got[1].q.src == 4);
    CHECK(pend.size() == 3 && pend[0].q.src == 1 && pend[1].q.src == 3 && pend[2].q.src == 5);
    got.clear();
    sched_take_bfs(pend, 0, 0, &got);
    CHECK(got.empty() && pend.size() == 3);
}

static void test_head_of_line_waits_for_memory() {
    // the oldest query does not fit: nothing is taken although a later one
    // would fit, and the queue is unchanged
    std::deque<PendingQ> pend = {q(1, GBGPU_QUERY_WBFS, 1), q(1, GBGPU_QUERY_BFS, 2)};
    ArenaAlloc a(256 * 200);
    std::vector<uint32_t> cap = {0, 0};
    std::vector<PendingQ> job;
    size_t off = 0, bytes = 0;
    uint32_t kc = 0;
    CHECK(!sched_admit(pend, a, fake_env({false, false}), cap, &job, &off, &bytes, &kc));
    CHECK(job.empty() && pend.size() == 2 && pend.front().q.src == 1);
    CHECK(a.largest() == 256 * 200);
    // once memory is released (a larger arena here) it runs
    ArenaAlloc b(256 * 1000);
    CHECK(sched_admit(pend, b, fake_env({false, false}), cap, &job, &off, &bytes, &kc));
    CHECK(job.size() == 1 && job[0].q.src == 1 && bytes == 256 * 364);
}

static void test_memory_accounting_over_a_run() {
    // admit until full, release, admit again: offsets never overlap
    std::deque<PendingQ> pend;
    for (int i = 0; i < 10; ++i) pend.push_back(q(1, GBGPU_QUERY_BFS, i));
    ArenaAlloc a(256 * 350);
    std::vector<uint32_t> cap = {0, 0};
    std::vector<PendingQ> job;
    std::vector<std::pair<size_t, size_t>> live;
    size_t off = 0, bytes = 0;
    uint32_t kc = 0;
    while (sched_admit(pend, a, fake_env({false, false}), cap, &job, &off, &bytes, &kc))
        live.emplace_back(off, bytes);
    CHECK(live.size() == 3 && pend.size() == 7);
    for (size_t i = 0; i < live.size(); ++i)
        for (size_t j = i + 1; j < live.size(); ++j)
            CHECK(live[i].first + live[i].second <= live[j].first ||
                  live[j].first + live[j].second <= live[i].first);
    a.release(live[1].first, live[1].second);
    CHECK(sched_admit(pend, a, fake_env({false, false}), cap, &job, &off, &bytes, &kc));
    CHECK(off == live[1].first);
}

static void test_learned_capacity_and_requeue() {
    SchedEnv env = fake_env({false, false});
    std::vector<uint32_t> cap = {0, 0};
    std::deque<PendingQ> pend = {q(1, GBGPU_QUERY_WBFS, 7), q(1, GBGPU_QUERY_BFS, 8)};
    ArenaAlloc a(256 * 100000);
    std::vector<PendingQ> job;
    size_t off = 0, bytes = 0;
    uint32_t kc = 0;
    CHECK(sched_admit(pend, a, env, cap, &job, &off, &bytes, &kc));
    CHECK(job.size() == 1 && job[0].cap == 0 && bytes == 256 * 364);
    // it overflowed capacity 64: back at the front with 128, one retry
    CHECK(sched_requeue_overflow(pend, env, cap, 256 * 100000, job[0], 64, 1000));
    CHECK(pend.size() == 2 && pend.front().q.src == 7 && pend.front().cap == 128 &&
          pend.front().retries == 1);
    CHECK(cap[1] == 128 && cap[0] == 0);
    // a later weighted query on the same graph starts from the learned 128
    pend.push_back(q(1, GBGPU_QUERY_WBFS, 9));
    a.release(off, bytes);
    CHECK(sched_admit(pend, a, env, cap, &job, &off, &bytes, &kc));  // the re-queued one
    CHECK(job[0].q.src == 7 && job[0].cap == 128);
    a.release(off, bytes);
    CHECK(sched_admit(pend, a, env, cap, &job, &off, &bytes, &kc));  // the BFS
    CHECK(job[0].q.src == 8 && job[0].cap == 0);
    a.release(off, bytes);
    CHECK(sched_admit(pend, a, env, cap, &job, &off, &bytes, &kc));
    CHECK(job[0].q.src == 9 && job[0].cap == 128 && job[0].retries == 0);
    // capacity doubles at most to n
    PendingQ big = job[0];
    CHECK(sched_requeue_overflow(pend, env, cap, 256 * 100000, big, 700, 1000));
    CHECK(pend.front().cap == 1000 && cap[1] == 1000);
    // a doubled workspace that can never fit fails the query instead
    std::deque<PendingQ> p2;
    CHECK(!sched_requeue_overflow(p2, env, cap, 256 * 400, big, 128, 1000));
    CHECK(p2.empty());
}

static void test_arena_random() {
    // random allocations against a unit bitmap
    const size_t units = 300;
    ArenaAlloc a(units * 256);
    std::vector<char> used(units, 0);
    std::vector<std::pair<size_t, size_t>> live;
    uint64_t x = 88172645463325252ull;
    auto rnd = [&]() { x ^= x << 13; x ^= x >> 7; x ^= x << 17; return x; };
    for (int i = 0; i < 20000; ++i) {
        if (live.empty() || rnd() % 3) {
            const size_t bytes = 1 + rnd() % (30 * 256);
            const size_t need = (bytes + 255) / 256;
            bool fit = false;
            for (size_t s0 = 0; s0 + need <= units && !fit; ++s0) {
                bool ok = true;
                for (size_t k = 0; k < need && ok; ++k) ok = !used[s0 + k];
                fit = ok;
            }
            size_t off = 0;
            const bool got = a.alloc(bytes, &off);
            CHECK(got == fit);
            if (got) {
                for (size_t k = 0; k < need; ++k) {
                    CHECK(!used[off / 256 + k]);
                    used[off / 256 + k] = 1;
                }
                live.emplace_back(off, bytes);
            }
        } else {
            const size_t j = rnd() % live.size();
            a.release(live[j].first, live[j].second);
            for (size_t k = 0; k < (live[j].second + 255) / 256; ++k) used[live[j].first / 256 + k] = 0;
            live.erase(live.begin() + (long)j);
        }
        if (failures) return;
    }
    for (auto& l : live) a.release(l.first, l.second);
    CHECK(a.largest() == units * 256);
}

// The learned capacity comes back down only after a full window of
// reports, only when it is at least four times the window's largest fill,
// and never below the default; unknown fills and the default are ignored.
static void test_learned_capacity_decay() {
    const uint32_t dflt = 1000;
    {
        uint32_t learned = 0;  // default: nothing to lower
        CapWindow w;
        for (uint32_t i = 0; i < 2 * kCapWindow; ++i) sched_note_peak(learned, w, 10, dflt);
        CHECK(learned == 0 && w.n == 0);
    }
    {
        uint32_t learned = 16000;  // an outlier grew it; later fills stay <= 3000
        CapWindow w;
        for (uint32_t i = 0; i + 1 < kCapWindow; ++i) sched_note_peak(learned, w, 500 + i * 80, dflt);
        CHECK(learned == 16000 && w.n == kCapWindow - 1);  // window not full yet
        sched_note_peak(learned, w, 0, dflt);               // unknown fill: not counted
        CHECK(learned == 16000 && w.n == kCapWindow - 1);
        sched_note_peak(learned, w, 3000, dflt);
        CHECK(learned == 6000 && w.n == 0);                  // twice the largest fill
    }
    {
        uint32_t learned = 16000;  // fills above a quarter of it: kept
        CapWindow w;
        for (uint32_t i = 0; i < kCapWindow; ++i) sched_note_peak(learned, w, i == 7 ? 4001 : 100, dflt);
        CHECK(learned == 16000 && w.n == 0);
    }
    {
        uint32_t learned = 4000;  // twice the largest fill is below the default
        CapWindow w;
        for (uint32_t i = 0; i < kCapWindow; ++i) sched_note_peak(learned, w, 300, dflt);
        CHECK(learned == 0);
    }
}

int main() {
    test_oldest_first_alone();
    test_packs_same_graph_bfs_in_order();
    test_pack_limit_and_halving();
    test_take_bfs_for_a_joining_round();
    test_head_of_line_waits_for_memory();
    test_memory_accounting_over_a_run();
    test_learned_capacity_and_requeue();
    test_learned_capacity_decay();
    test_arena_random();
    if (failures) {
        printf("%d checks failed\n", failures);
        return 1;
    }
    printf("scheduler checks passed\n");
    return 0;
}
