// Host-side scheduling rules of the query server: the first-fit arena
// allocator, the pending-query record, the admission rule (which pending
// queries the next free worker takes) and the rule applied after a weighted
// query overflowed its distance buckets.  Plain C++ with no HIP dependency,
// so the rules are unit-tested on the CPU (under address and
// undefined-behaviour sanitizers) with fake graphs and footprints.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <algorithm>
#include <deque>
#include <functional>
#include <iterator>
#include <map>
#include <vector>

#include "gbgpu.h"

namespace gb {

// First-fit allocator over [0, size) in 256-byte units, with coalescing of
// free ranges.
class ArenaAlloc {
  public:
    explicit ArenaAlloc(size_t size) { if (size) free_[0] = size; }
    bool alloc(size_t bytes, size_t* off) {
        bytes = (bytes + 255) & ~(size_t)255;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes;
                const size_t noff = it->first + bytes;
                free_.erase(it);
                if (rest) free_[noff] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = (bytes + 255) & ~(size_t)255;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t largest() const {
        size_t m = 0;
        for (auto& kv : free_) m = std::max(m, kv.second);
        return m;
    }

  private:
    std::map<size_t, size_t> free_;
};

struct PendingQ {
    uint64_t ticket;
    gbgpu_query q;
    int64_t t_arrive;
    uint32_t cap;        // weighted BFS bucket capacity override (0 = default)
    int32_t retries;     // runs repeated after a bucket overflow
    int64_t t_start;     // when it joined a running group (0: with the run)
    int32_t join_round;  // round of the running group it joined before
};

// Largest graph whose same-graph BFS queries are bit-packed together, and
// the most queries one packed run takes (one 64-bit mask per vertex).
constexpr int64_t kPackedMaxN = 1 << 24;
constexpr int kPackedMaxK = 64;

// What the admission rule needs to know of the server's graphs and
// workspaces (the server binds these to its graph handles; the unit tests
// to fakes).
struct SchedEnv {
    // graph may bit-pack its BFS queries (shallow and small enough)
    std::function<bool(int32_t gid)> packable;
    // device bytes of one query of `kind` with bucket capacity override cap
    std::function<size_t(int32_t gid, int32_t kind, uint32_t cap)> footprint;
    // device bytes of a bit-packed run of k BFS queries
    std::function<size_t(int32_t gid, int64_t k)> packed_bytes;
};

// Takes the first k pending BFS queries on graph gid (in their order).
inline void sched_take_bfs(std::deque<PendingQ>& pending, int32_t gid, int k,
                           std::vector<PendingQ>* out) {
    for (auto it = pending.begin(); it != pending.end() && (int)out->size() < k;) {
        if (it->q.kind == GBGPU_QUERY_BFS && it->q.graph_id == gid) {
            out->push_back(*it);
            it = pending.erase(it);
        } else {
            ++it;
        }
    }
}

// Admission: looks at the oldest pending query.  A BFS on a packable graph
// takes, with it, the other pending BFS queries on the same graph (oldest
// first, up to kPackedMaxK): as a group with room for kPackedMaxK sources
// when that workspace fits (*kcap = kPackedMaxK: later BFS arrivals on the
// graph may join it at a round boundary), else as the largest group whose
// workspace fits, halving the group size from all of them down to 2
// (*kcap = its size); otherwise the oldest query runs alone if its
// footprint fits (a weighted query with the bucket capacity an earlier
// query on its graph grew to, from learned_cap; *kcap = 0); otherwise
// nothing is taken and the worker waits for memory (later queries do not
// overtake the oldest).  On success the taken queries leave `pending` in
// their order, `off`/`bytes` hold the workspace in the arena.
inline bool sched_admit(std::deque<PendingQ>& pending, ArenaAlloc& alloc, const SchedEnv& env,
                        const std::vector<uint32_t>& learned_cap, std::vector<PendingQ>* job,
                        size_t* off, size_t* bytes, uint32_t* kcap) {
    job->clear();
    *kcap = 0;
    if (pending.empty()) return false;
    const PendingQ& head = pending.front();
    const int32_t gid = head.q.graph_id;
    int nsame = 0;
    if (head.q.kind == GBGPU_QUERY_BFS && env.packable(gid))
        for (auto& p : pending)
            if (p.q.kind == GBGPU_QUERY_BFS && p.q.graph_id == gid && nsame < kPackedMaxK) ++nsame;
    if (nsame > 1) {
        const size_t bb = env.packed_bytes(gid, kPackedMaxK);
        if (alloc.alloc(bb, off)) {
            *bytes = bb;
            *kcap = kPackedMaxK;
            sched_take_bfs(pending, gid, nsame, job);
            return true;
        }
    }
    for (int kb = nsame; kb > 1; kb /= 2) {
        const size_t bb = env.packed_bytes(gid, kb);
        if (alloc.alloc(bb, off)) {
            *bytes = bb;
            *kcap = (uint32_t)kb;
            sched_take_bfs(pending, gid, kb, job);
            return true;
        }
    }
    const uint32_t cap = head.cap ? head.cap
                       : head.q.kind == GBGPU_QUERY_WBFS ? learned_cap[gid] : 0u;
    const size_t nb = env.footprint(gid, head.q.kind, cap);
    if (alloc.alloc(nb, off)) {
        *bytes = nb;
        job->push_back(head);
        job->back().cap = cap;
        pending.pop_front();
        return true;
    }
    return false;
}

// After a weighted query's run overflowed its buckets (capacity C, graph of
// n vertices): it goes back to the front of the queue with twice the
// capacity (at most n) and one more retry, and the graph's learned capacity
// grows to that; if the doubled workspace could never fit in the arena the
// query fails instead (returns false: finish it with E_NOMEM).
inline bool sched_requeue_overflow(std::deque<PendingQ>& pending, const SchedEnv& env,
                                   std::vector<uint32_t>& learned_cap, size_t arena_bytes,
                                   const PendingQ& q, uint32_t C, int64_t n) {
    const uint32_t newcap = (uint32_t)std::min<int64_t>(n, (int64_t)C * 2);
    if (env.footprint(q.q.graph_id, GBGPU_QUERY_WBFS, newcap) > arena_bytes) return false;
    PendingQ p = q;
    p.cap = newcap;
    p.retries += 1;
    uint32_t& learned = learned_cap[p.q.graph_id];
    learned = std::max(learned, newcap);
    pending.push_front(p);
    return true;
}

// The learned bucket capacity of a graph coming back down.  Every weighted
// query on the graph that finished without overflow reports the fill of its
// fullest bucket (`peak`; 0 when unknown).  Once kCapWindow such reports
// have been seen, a learned capacity at least four times the largest of
// them drops to twice that largest fill, or back to the default (0) when
// that is not above default_cap; then a new window starts.  One outlier
// source that forced the capacity up thus stops inflating every later
// query's footprint, and a graph whose queries keep filling their buckets
// keeps its capacity.
constexpr uint32_t kCapWindow = 32;

struct CapWindow {
    uint32_t peak_max = 0;
    uint32_t n = 0;
};

inline void sched_note_peak(uint32_t& learned, CapWindow& w, uint32_t peak,
                            uint32_t default_cap) {
    if (learned == 0 || peak == 0) return;  // nothing learned, or fill unknown
    w.peak_max = std::max(w.peak_max, peak);
    if (++w.n < kCapWindow) return;
    if ((uint64_t)w.peak_max * 4 <= (uint64_t)learned) {
        const uint64_t c = (uint64_t)w.peak_max * 2;
        learned = c <= default_cap ? 0u : (uint32_t)c;
    }
    w = CapWindow{};
}

}  // namespace gb
