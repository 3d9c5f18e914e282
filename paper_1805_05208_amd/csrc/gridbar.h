// Grid-wide barrier for kernels launched cooperatively (every workgroup
// resident), used by the single-launch forms of the BFS and batched BFS
// rounds.  The caller provides kBarWords 32-bit words of device memory,
// zeroed before the launch.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace gb {

constexpr int kBarWords = 4096;

// Layout of the barrier area (32-bit words; fields that
// different workgroups update sit 256 bytes apart):
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
// barrier number, from 1), so nothing is reset between barriers.  A wait longer than kBarrierSpin polls
// sets the abort word and gives up; every wait also gives up once the abort
// word is set, so the kernel always ends and the host can fall back.
constexpr uint64_t kBarrierSpin = 1ull << 22;

struct DieInfo {
    uint32_t die, nwg, ndies;  // this workgroup's die, workgroups on it, dies in use
};

__device__ __forceinline__ uint32_t bar_ld(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void bar_st(uint32_t* p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t bar_add(uint32_t* p) {
    return __hip_atomic_fetch_add(p, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1u;
}

// Polls *p until it equals want (relaxed device-scope loads: an acquire load
// would invalidate the caches at every poll).  False when the abort word is
// set or the wait gave up.
__device__ __forceinline__ bool bar_wait(const uint32_t* p, uint32_t want, uint32_t* bar) {
    uint64_t spins = 0;
    while (bar_ld(p) != want) {
        if (bar_ld(bar + kBarAbort)) return false;
        if (++spins > kBarrierSpin) {
            bar_st(bar + kBarAbort, 1u);
            return false;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    return true;
}

// The die (XCD) this wave runs on, from the hardware register.
__device__ __forceinline__ uint32_t die_id() {
    uint32_t x;
    asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(x));
    return x & (kBarMaxDies - 1);
}

// Start-up census (all workgroups, once): counts the workgroups of each die
// behind one plain counting barrier.
__device__ bool bar_census(uint32_t* bar, DieInfo& di) {
    __shared__ uint32_t s_ok;
    if (threadIdx.x == 0) {
        const uint32_t x = die_id();
        __hip_atomic_fetch_add(bar + kBarDieCount + kBarDieStride * x, 1u, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        bool ok = true;
        if (bar_add(bar + kBarCensusCnt) == gridDim.x) {
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
            bar_st(bar + kBarCensusDone, 1u);
        } else {
            ok = bar_wait(bar + kBarCensusDone, 1u, bar);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        uint32_t nd = 0;
        for (uint32_t d = 0; d < (uint32_t)kBarMaxDies; ++d)
            nd += bar_ld(bar + kBarDieCount + kBarDieStride * d) ? 1u : 0u;
        di.die = x;
        di.nwg = bar_ld(bar + kBarDieCount + kBarDieStride * x);
        di.ndies = nd;
        s_ok = ok ? 1u : 0u;
    }
    __syncthreads();
    return s_ok != 0u;
}

// Barrier number e (from 1).  Returns false when the kernel must stop.
__device__ __forceinline__ bool grid_barrier(uint32_t* bar, const DieInfo& di, uint32_t e) {
    __shared__ uint32_t s_ok;
    // every wave's stores complete (in the die's L2) before the arrival
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        bool ok = true;
        uint32_t* release = bar + kBarDieRelease + kBarDieStride * di.die;
        if (bar_add(bar + kBarDieArrive + kBarDieStride * di.die) == e * di.nwg) {
            // die leader: the die's stores go to memory, then the leaders meet
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            if (bar_add(bar + kBarLeaders) == e * di.ndies) {
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
                bar_st(bar + kBarGen, e);
            } else {
                ok = bar_wait(bar + kBarGen, e, bar);
            }
            // one invalidate of the die's L2 (and this CU's L1), finished
            // before the die is released
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            __builtin_amdgcn_s_waitcnt(0);
            if (ok) bar_st(release, e);
        } else {
            ok = bar_wait(release, e, bar);
            // a workgroup-scope invalidate need not drop this CU's L1 lines,
            // so each workgroup takes the device-scope acquire itself
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        s_ok = ok ? 1u : 0u;
    }
    __syncthreads();
    return s_ok != 0u;
}

}  // namespace gb
