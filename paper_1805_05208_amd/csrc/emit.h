// Workgroup-level output compaction for frontier kernels.
//
// The paper's edgeMapBlocked packs each block's live neighbours, prefix-sums
// the per-block counts and compacts them (no separate filter pass).  Here a
// block is one workgroup: wavefronts append newly reached vertices to an LDS
// buffer with a ballot + popcount slot, and at the end of the launch the
// workgroup reserves its range of the output queue with ONE packed 64-bit
// atomicAdd (count << 32 | sum of degrees) and writes ids and exclusive degree
// prefix sums with a workgroup scan.  Same-address device atomics serialise
// (one every ~12 ns on this part), so reservations per workgroup rather than
// per wavefront keep a round's fixed cost low.  Round totals go to 32
// counters on separate cache lines.
#pragma once

#include "common.h"

namespace gb {

constexpr int kRBlock = 1024;               // threads per traversal workgroup
constexpr int kRWaves = kRBlock / kWave;    // 16 wavefronts
constexpr int kWgCap = 8192;                // LDS entries per workgroup
constexpr int kSpread = 32;                 // spread total counters
constexpr int kSpreadStride = 16;           // u64 per counter (128 B apart)

// Output queue of one round: ids Q, exclusive degree prefix P, packed
// reservation counter, abandon flag and limit.
struct QueueOut {
    uint32_t* Q;
    uint32_t* P;
    unsigned long long* qcnt;
    unsigned long long* qover;
    uint64_t qlimit;
    unsigned long long* tot;  // kSpread counters, kSpreadStride apart
};

struct WgQueue {
    uint32_t v[kWgCap];
    uint32_t d[kWgCap];
    uint32_t cnt;
    uint32_t dsum;
    uint32_t found;
    uint32_t fdsum;
    unsigned long long base;
    uint32_t wsum[kRWaves];
};

__device__ __forceinline__ void wgq_init(WgQueue& q) {
    if (threadIdx.x == 0) {
        q.cnt = 0;
        q.dsum = 0;
        q.found = 0;
        q.fdsum = 0;
    }
}

// Sum of the kSpread counters (called by one full wavefront).
__device__ __forceinline__ unsigned long long spread_sum(const unsigned long long* tot) {
    const int l = lane_id();
    unsigned long long x = l < kSpread ? tot[l * kSpreadStride] : 0ull;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        uint32_t lo = __shfl_xor((uint32_t)x, d, 64);
        uint32_t hi = __shfl_xor((uint32_t)(x >> 32), d, 64);
        x += ((unsigned long long)hi << 32) | lo;
    }
    return x;
}

// Writes lanes' (v, dv) straight to the output queue (used when the LDS
// buffer is full).  Wave-uniform call.
__device__ __forceinline__ void wave_direct_emit(bool take, uint32_t v, uint32_t dv, uint64_t m,
                                                 const QueueOut& out) {
    const int l = lane_id();
    const uint32_t k = (uint32_t)__popcll(m);
    const uint32_t x = take ? dv : 0u;
    const uint32_t inc = wave_incl_sum(x);
    const uint32_t ds = __shfl(inc, 63, 64);
    const int ld = first_lane(m);
    unsigned long long packed = ~0ull;
    if (l == ld && *(volatile unsigned long long*)out.qover == 0) {
        packed = atomicAdd(out.qcnt, ((unsigned long long)k << 32) | ds);
        if ((uint64_t)(packed >> 32) + k + (uint32_t)packed + ds > out.qlimit) {
            *out.qover = 1ull;
            packed = ~0ull;
        }
    }
    packed = shfl64(packed, ld);
    if (packed != ~0ull && take) {
        const uint32_t pos = (uint32_t)(packed >> 32) + mbcnt(m);
        out.Q[pos] = v;
        out.P[pos] = (uint32_t)packed + inc - x;
    }
}

// Wave-uniform: counts the lanes with `take` set in the round totals only.
__device__ __forceinline__ void wgq_count(WgQueue& q, bool take, uint32_t dv) {
    const uint64_t m = ballot(take);
    if (!m) return;
    const uint32_t ds = wave_sum(take ? dv : 0u);
    if (lane_id() == first_lane(m)) {
        atomicAdd(&q.found, (uint32_t)__popcll(m));
        atomicAdd(&q.fdsum, ds);
    }
}

// Wave-uniform: appends the lanes with `take` set.
__device__ __forceinline__ void wgq_push(WgQueue& q, bool take, uint32_t v, uint32_t dv,
                                         const QueueOut& out) {
    const uint64_t m = ballot(take);
    if (!m) return;
    const int l = lane_id();
    const uint32_t k = (uint32_t)__popcll(m);
    const uint32_t ds = wave_sum(take ? dv : 0u);
    const int ld = first_lane(m);
    uint32_t pos0 = kNone;
    if (l == ld) {
        atomicAdd(&q.found, k);
        atomicAdd(&q.fdsum, ds);
        uint32_t old = *(volatile uint32_t*)&q.cnt;
        for (;;) {
            if (old + k > (uint32_t)kWgCap) break;
            uint32_t prev = atomicCAS(&q.cnt, old, old + k);
            if (prev == old) {
                pos0 = old;
                break;
            }
            old = prev;
        }
        if (pos0 != kNone) atomicAdd(&q.dsum, ds);
    }
    pos0 = __shfl(pos0, ld, 64);
    if (pos0 != kNone) {
        if (take) {
            const uint32_t i = pos0 + mbcnt(m);
            q.v[i] = v;
            q.d[i] = dv;
        }
    } else {
        wave_direct_emit(take, v, dv, m, out);
    }
}

// Workgroup-uniform: one reservation for the buffered entries, then a
// workgroup scan writes ids and degree prefix sums; the buffer is emptied.
__device__ __forceinline__ void wgq_flush(WgQueue& q, const QueueOut& out, bool emit_queue) {
    __syncthreads();
    const uint32_t n = q.cnt;
    __syncthreads();  // every thread has read n before anyone can append again
    if (n == 0) return;  // workgroup-uniform
    if (threadIdx.x == 0) {
        unsigned long long packed = ~0ull;
        if (emit_queue && *(volatile unsigned long long*)out.qover == 0) {
            packed = atomicAdd(out.qcnt, ((unsigned long long)n << 32) | q.dsum);
            if ((uint64_t)(packed >> 32) + n + (uint32_t)packed + q.dsum > out.qlimit) {
                *out.qover = 1ull;
                packed = ~0ull;
            }
        }
        q.base = packed;
    }
    __syncthreads();
    const unsigned long long base = q.base;
    if (base != ~0ull) {  // workgroup-uniform
        const int t = threadIdx.x;
        const int l = lane_id();
        const int wv = t / kWave;
        constexpr int PER = kWgCap / kRBlock;
        uint32_t loc[PER];
        uint32_t s = 0;
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const uint32_t idx = (uint32_t)(PER * t + i);
            const uint32_t x = idx < n ? q.d[idx] : 0u;
            loc[i] = s;
            s += x;
        }
        const uint32_t inc = wave_incl_sum(s);
        if (l == 63) q.wsum[wv] = inc;
        __syncthreads();
        if (t < kWave) {
            const uint32_t x = t < kRWaves ? q.wsum[t] : 0u;
            const uint32_t c = wave_incl_sum(x);
            if (t < kRWaves) q.wsum[t] = c - x;
        }
        __syncthreads();
        const uint32_t off = q.wsum[wv] + inc - s;
        const uint32_t c0 = (uint32_t)(base >> 32);
        const uint32_t e0 = (uint32_t)base;
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const uint32_t idx = (uint32_t)(PER * t + i);
            if (idx < n) {
                out.Q[c0 + idx] = q.v[idx];
                out.P[c0 + idx] = e0 + off + loc[i];
            }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        q.cnt = 0;
        q.dsum = 0;
    }
    __syncthreads();
}

// Workgroup-uniform: flush when fewer than `room` free entries remain.
__device__ __forceinline__ void wgq_maybe_flush(WgQueue& q, const QueueOut& out, bool emit_queue,
                                                uint32_t room) {
    __syncthreads();
    const uint32_t n = q.cnt;
    __syncthreads();  // a uniform decision: every thread read the same n
    if (n + room > (uint32_t)kWgCap) wgq_flush(q, out, emit_queue);
}

// Workgroup-uniform, at the end of the launch: flush, then add the
// workgroup's totals to a spread counter.
__device__ __forceinline__ void wgq_finish(WgQueue& q, const QueueOut& out, bool emit_queue) {
    wgq_flush(q, out, emit_queue);
    if (threadIdx.x == 0 && q.found)
        atomicAdd(&out.tot[(blockIdx.x % kSpread) * kSpreadStride],
                  ((unsigned long long)q.found << 32) | q.fdsum);
}

}  // namespace gb
