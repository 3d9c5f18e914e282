// Grid-wide barrier for kernels launched cooperatively (every workgroup
// resident), used by the single-launch forms of the BFS and batched BFS
// rounds: the protocol of gridbar_protocol.h on the device.  The caller
// provides kBarWords 32-bit words of device memory, zeroed before the
// launch.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "gridbar_protocol.h"

namespace gb {

constexpr uint64_t kBarrierSpin = 1ull << 22;

// Device memory operations of the protocol: relaxed device-scope atomics,
// device-scope fences, s_waitcnt, s_sleep.
struct DevMem {
    static constexpr uint64_t kSpin = kBarrierSpin;
    __device__ static __forceinline__ uint32_t ld(const uint32_t* p) {
        return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __device__ static __forceinline__ void st(uint32_t* p, uint32_t v) {
        __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __device__ static __forceinline__ uint32_t add(uint32_t* p) {
        return __hip_atomic_fetch_add(p, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1u;
    }
    __device__ static __forceinline__ void release() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); }
    __device__ static __forceinline__ void acquire() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }
    __device__ static __forceinline__ void acq_rel() { __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent"); }
    __device__ static __forceinline__ void settle() { __builtin_amdgcn_s_waitcnt(0); }
    __device__ static __forceinline__ void pause() { __builtin_amdgcn_s_sleep(1); }
};

// The die (XCD) this wave runs on, from the hardware register.
__device__ __forceinline__ uint32_t die_id() {
    uint32_t x;
    asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(x));
    return x & (kBarMaxDies - 1);
}

// Start-up census, by thread 0 of every workgroup; the result is shared
// with the workgroup.
__device__ bool bar_census(uint32_t* bar, DieInfo& di) {
    __shared__ uint32_t s_ok;
    if (threadIdx.x == 0) s_ok = bar_census_core<DevMem>(bar, die_id(), gridDim.x, di) ? 1u : 0u;
    __syncthreads();
    return s_ok != 0u;
}

// Barrier number e (from 1).  Every wave's stores complete (in the die's
// L2) before the workgroup barrier; thread 0 then runs the protocol.
// Returns false when the kernel must stop.
__device__ __forceinline__ bool grid_barrier(uint32_t* bar, const DieInfo& di, uint32_t e) {
    __shared__ uint32_t s_ok;
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) s_ok = grid_barrier_core<DevMem>(bar, di, e) ? 1u : 0u;
    __syncthreads();
    return s_ok != 0u;
}

}  // namespace gb
