// Wave-level pieces of the persistent scheduler, shared by the DFS kernels of
// every search (nq_dfs_kernel, nq_perm_kernel).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace nqi {

// Rank of this lane among the set lanes of `mask` (lanes below it).
__device__ __forceinline__ uint32_t lane_rank(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ uint64_t shfl_u64(uint64_t v, int src) {
    uint32_t lo = __shfl((int)(uint32_t)v, src, 64);
    uint32_t hi = __shfl((int)(uint32_t)(v >> 32), src, 64);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int mask) {
    uint32_t lo = __shfl_xor((int)(uint32_t)v, mask, 64);
    uint32_t hi = __shfl_xor((int)(uint32_t)(v >> 32), mask, 64);
    return ((uint64_t)hi << 32) | lo;
}

// One scheduler visit's refill of a persistent launch.  The wave's share of
// the work queue is wave-uniform state kept by the caller: the entries
// [qlo, qhi) it has claimed and not yet handed out, whether the shared head
// has passed the end (claimed_all) and whether nothing is left to take
// (exhausted).  The idle lanes (no entry held) take, in rank order, the
// wave's unused claimed entries first, then a fresh block of at least
// `claim` entries claimed by the first idle lane with one atomic add on
// `head`; take(i) is called by each lane that gets entry i.  Entries at or
// past `len` are never handed out.  Every lane of the wave calls it.
template <class Take>
__device__ __forceinline__ void refill_idle_lanes(uint64_t& qlo, uint64_t& qhi, bool& claimed_all,
                                                  bool& exhausted, bool has_task, uint32_t lane,
                                                  unsigned long long* head, uint64_t len,
                                                  uint32_t claim, Take&& take) {
    const uint64_t idle = __ballot(!has_task);
    if (idle != 0) {
        const uint32_t want = (uint32_t)__popcll(idle);
        const uint64_t have = qhi - qlo;
        uint64_t nlo = 0, nhi = 0;
        if (have < want && !claimed_all) {
            const uint64_t grab = max((uint64_t)(want - have), (uint64_t)claim);
            const int leader = __ffsll((unsigned long long)idle) - 1;
            uint64_t first = 0;
            if ((int)lane == leader) first = atomicAdd(head, (unsigned long long)grab);
            first = shfl_u64(first, leader);
            nlo = min(first, len);
            nhi = min(first + grab, len);
            if (first + grab >= len) claimed_all = true;
        }
        if (!has_task) {
            const uint64_t rk = lane_rank(idle);
            if (rk < have) take(qlo + rk);
            else if (nlo + (rk - have) < nhi) take(nlo + (rk - have));
        }
        if (want <= have) {
            qlo += want;
        } else {
            qlo = min(nlo + (want - have), nhi);
            qhi = nhi;
        }
        if (claimed_all && qlo >= qhi) exhausted = true;
    }
}

}  // namespace nqi
