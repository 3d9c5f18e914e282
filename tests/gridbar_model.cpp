// Host model of the grid-barrier protocol of the single-launch forms
// (gridbar_protocol.h): the same census and barrier code, instantiated with
// memory operations on threads (GCC atomics on the same barrier words,
// fences, yield), run by threads standing for workgroups spread unevenly
// over dies.  Checks that every barrier completes, that after barrier e
// every thread sees every other thread's store of epoch e, that the census
// counts the workgroups of each die and the dies in use, and that when one
// thread stops arriving every other wait gives up (abort word set) instead
// of hanging.  Built and run under address and undefined-behaviour
// sanitizers by test_host_sanitized.py; prints one line per failed check.
#define __device__
#define __forceinline__ inline
#include "gridbar_protocol.h"

#include <stdio.h>

#include <thread>
#include <vector>

using namespace gb;

struct HostMem {
    static constexpr uint64_t kSpin = 1ull << 16;
    static uint32_t ld(const uint32_t* p) { return __atomic_load_n(p, __ATOMIC_RELAXED); }
    static void st(uint32_t* p, uint32_t v) { __atomic_store_n(p, v, __ATOMIC_RELAXED); }
    static uint32_t add(uint32_t* p) { return __atomic_add_fetch(p, 1u, __ATOMIC_RELAXED); }
    static void release() { __atomic_thread_fence(__ATOMIC_RELEASE); }
    static void acquire() { __atomic_thread_fence(__ATOMIC_ACQUIRE); }
    static void acq_rel() { __atomic_thread_fence(__ATOMIC_ACQ_REL); }
    static void settle() {}
    static void pause() { std::this_thread::yield(); }
};

static int failures = 0;
#define CHECK(cond)                                                        \
    do {                                                                   \
        if (!(cond)) {                                                     \
            printf("FAIL %s:%d: %s\n", __FILE__, __LINE__, #cond);         \
            __atomic_add_fetch(&failures, 1, __ATOMIC_RELAXED);            \
        }                                                                  \
    } while (0)

// n threads on the given dies run `epochs` barriers; thread `quitter` (if
// >= 0) stops before barrier quit_at.  Each epoch a thread writes its slot
// of the epoch's parity and, after the barrier, reads every slot.
static void run(const std::vector<uint32_t>& dies, uint32_t epochs, int quitter, uint32_t quit_at) {
    const uint32_t n = (uint32_t)dies.size();
    std::vector<uint32_t> bar(kBarWords, 0u);
    std::vector<uint32_t> data(2 * n, 0u);
    uint32_t nd = 0;
    for (uint32_t d = 0; d < (uint32_t)kBarMaxDies; ++d) {
        bool used = false;
        for (uint32_t x : dies) used |= x == d;
        nd += used ? 1u : 0u;
    }
    std::vector<std::thread> th;
    for (uint32_t t = 0; t < n; ++t) {
        th.emplace_back([&, t]() {
            DieInfo di{};
            CHECK(bar_census_core<HostMem>(bar.data(), dies[t], n, di));
            uint32_t same = 0;
            for (uint32_t x : dies) same += x == dies[t] ? 1u : 0u;
            CHECK(di.die == dies[t] && di.nwg == same && di.ndies == nd);
            for (uint32_t e = 1; e <= epochs; ++e) {
                if ((int)t == quitter && e == quit_at) return;
                data[(e & 1u) * n + t] = e * 1000u + t;
                const bool ok = grid_barrier_core<HostMem>(bar.data(), di, e);
                if (quitter >= 0 && e >= quit_at) {
                    CHECK(!ok);  // someone stopped arriving: the wait gave up
                    return;
                }
                CHECK(ok);
                if (!ok) return;
                for (uint32_t u = 0; u < n; ++u) CHECK(data[(e & 1u) * n + u] == e * 1000u + u);
            }
        });
    }
    for (auto& x : th) x.join();
    if (quitter >= 0) CHECK(HostMem::ld(&bar[kBarAbort]) == 1u);
    else CHECK(HostMem::ld(&bar[kBarAbort]) == 0u && HostMem::ld(&bar[kBarGen]) == epochs);
}

int main() {
    run({0, 0, 0, 1, 1, 2, 5, 5, 5, 5, 7, 15}, 300, -1, 0);  // uneven dies, gaps
    run({3}, 50, -1, 0);                                       // one workgroup
    run({0, 1, 2, 3, 4, 5, 6, 7}, 200, -1, 0);                 // one per die
    run({0, 0, 1, 1, 2, 2}, 20, 4, 7);                         // a workgroup stops
    if (failures) {
        printf("%d checks failed\n", failures);
        return 1;
    }
    printf("grid barrier model checks passed\n");
    return 0;
}
