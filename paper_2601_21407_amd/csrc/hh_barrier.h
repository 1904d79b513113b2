// hh_barrier.h -- grid-wide barrier of the persistent (cooperative) kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hhk {

// Grid barrier over co-resident blocks on a monotonic arrival counter: the
// g-th barrier of a launch is passed once the counter reaches
// (g + 1) * nblocks, so nobody has to reset it and a waiting block needs
// only the arrivals, not a second store from the last arriver.  Data
// shared across blocks (the arrival accumulators) is only touched by
// device-scope atomics, so most lanes need ordering, not cache maintenance:
// every wavefront waits for its own memory operations to complete, the
// block synchronizes, and one lane publishes the block's writes device-wide
// (release on its arrival), polls the counter with device-scope relaxed
// loads -- no cache invalidation per poll -- and performs one acquire fence
// when it is complete.  Every wait is bounded: after spin_limit polls the
// block flags a timeout, and any block that sees the flag leaves the time
// loop, so the grid always drains.
__device__ bool grid_barrier(unsigned* bar, unsigned nblocks, unsigned& gen, uint32_t spin_limit,
                             int32_t* flags, int* s_ok) {
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned target = (gen + 1) * nblocks;
    int ok = 1;
    unsigned seen =
        __hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT) + 1u;
    uint32_t spins = 0;
    while ((int)(seen - target) < 0) {
      if (++spins > spin_limit) {
        ok = 0;
        __hip_atomic_fetch_or(&flags[1], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
      seen = __hip_atomic_load(&bar[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (__hip_atomic_load(&flags[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) ok = 0;
    gen = gen + 1;
    *s_ok = ok;
  }
  __syncthreads();
  return *s_ok != 0;
}

}  // namespace hhk
