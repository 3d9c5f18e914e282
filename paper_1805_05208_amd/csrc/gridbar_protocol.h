// Grid-barrier protocol of the single-launch forms, run by one thread of
// every workgroup: the start-up census and barrier number e.  It is written
// against a policy M of memory operations on the barrier words -- ld / st /
// add (relaxed, device scope; add returns the new value), release /
// acquire / acq_rel fences, settle (wait for this thread's outstanding
// memory operations), pause, and kSpin (polls before a wait gives up) -- so
// that the same code runs on the device (gridbar.h) and in a host model test
// on threads (tests/gridbar_model.cpp).
#pragma once

#include <cstdint>

namespace gb {

constexpr int kBarWords = 4096;

// Layout of the barrier area (32-bit words; fields that different
// workgroups update sit 256 bytes apart):
//   [0]   arrivals at the start-up census     [64]  census done
//   [128] abort word                          [192] arrivals of die leaders
//   [256] generation (last finished barrier)
//   [512 + 64 x]  workgroups resident on die x (x < 16)
//   [1536 + 64 x] arrivals on die x           [2560 + 64 x] release of die x
constexpr int kBarCensusCnt = 0, kBarCensusDone = 64, kBarAbort = 128, kBarLeaders = 192,
              kBarGen = 256, kBarDieCount = 512, kBarDieArrive = 1536, kBarDieRelease = 2560,
              kBarDieStride = 64, kBarMaxDies = 16;
// words from kBarUser on are the caller's (cleared with the rest)
constexpr int kBarUser = kBarDieRelease + kBarMaxDies * kBarDieStride;
static_assert(kBarUser + 64 <= kBarWords, "barrier area");

// The barrier.  CDNA keeps one L2 per die (XCD), and the device-scope
// fences that make stores visible across dies write back (release) or
// invalidate (acquire) that whole L2.  So the workgroups of each die elect
// a leader per barrier, the last of them to arrive, which alone writes the
// die's L2 back and meets the other dies' leaders, then releases its die;
// every workgroup takes its own acquire (an invalidate of narrower scope
// need not drop the CU's L1 lines).  Every count is monotone (epoch e =
// barrier number, from 1), so nothing is reset between barriers.  A wait
// longer than M::kSpin polls sets the abort word and gives up; every wait
// also gives up once the abort word is set, so the kernel always ends and
// the host can fall back.
struct DieInfo {
    uint32_t die, nwg, ndies;  // this workgroup's die, workgroups on it, dies in use
};

// Polls *p until it equals want (relaxed loads: on the device an acquire
// load would invalidate the caches at every poll).  False when the abort
// word is set or the wait gave up (then it sets the abort word).
template <class M>
__device__ __forceinline__ bool bar_wait(const uint32_t* p, uint32_t want, uint32_t* bar) {
    uint64_t spins = 0;
    while (M::ld(p) != want) {
        if (M::ld(bar + kBarAbort)) return false;
        if (++spins > M::kSpin) {
            M::st(bar + kBarAbort, 1u);
            return false;
        }
        M::pause();
    }
    return true;
}

// Start-up census (every workgroup once, before the first barrier):
// workgroups per die behind one plain counting barrier.  `die` is the
// caller's die, `nblocks` the number of workgroups.
template <class M>
__device__ __forceinline__ bool bar_census_core(uint32_t* bar, uint32_t die, uint32_t nblocks,
                                                DieInfo& di) {
    M::add(bar + kBarDieCount + kBarDieStride * die);
    M::release();
    bool ok = true;
    if (M::add(bar + kBarCensusCnt) == nblocks) {
        M::acq_rel();
        M::st(bar + kBarCensusDone, 1u);
    } else {
        ok = bar_wait<M>(bar + kBarCensusDone, 1u, bar);
    }
    M::acquire();
    uint32_t nd = 0;
    for (uint32_t d = 0; d < (uint32_t)kBarMaxDies; ++d)
        nd += M::ld(bar + kBarDieCount + kBarDieStride * d) ? 1u : 0u;
    di.die = die;
    di.nwg = M::ld(bar + kBarDieCount + kBarDieStride * die);
    di.ndies = nd;
    return ok;
}

// Barrier number e (from 1), after the caller's workgroup has finished its
// stores.  Returns false when the kernel must stop.
template <class M>
__device__ __forceinline__ bool grid_barrier_core(uint32_t* bar, const DieInfo& di, uint32_t e) {
    bool ok = true;
    uint32_t* release = bar + kBarDieRelease + kBarDieStride * di.die;
    if (M::add(bar + kBarDieArrive + kBarDieStride * di.die) == e * di.nwg) {
        // die leader: the die's stores go to memory, then the leaders meet
        M::release();
        if (M::add(bar + kBarLeaders) == e * di.ndies) {
            M::acq_rel();
            M::st(bar + kBarGen, e);
        } else {
            ok = bar_wait<M>(bar + kBarGen, e, bar);
        }
        // the acquire (on the device: one invalidate of the die's L2 and
        // this CU's L1) is finished before the die is released
        M::acquire();
        M::settle();
        if (ok) M::st(release, e);
    } else {
        ok = bar_wait<M>(release, e, bar);
        // a narrower-scope invalidate need not drop the CU's L1 lines, so
        // each workgroup takes the acquire itself
        M::acquire();
    }
    return ok;
}

}  // namespace gb
