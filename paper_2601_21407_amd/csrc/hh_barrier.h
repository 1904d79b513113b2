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

// Flag-array variant: every block stores its arrival (the generation it
// reached) into a slot of its own, with release; wavefront 0 of block 0
// reads all the slots, 64 per load instruction, until every block has
// arrived, then releases the grid through eight flags on separate lines
// (block b polls flag b mod 8).  No read-modify-write is contended, so the
// cost grows much more slowly with the grid than the single counter's
// (measured: 10.5 against 19.0 us per barrier at 446 blocks; packed slots
// were faster than one 128-byte line per slot, 12.5 us, and a two-level
// counter tree slower, 11.6-16.6 us with 8-64 groups).  bar[32 g] for g < 8:
// release flags; bar[256 + b]: arrival slots; 256 + nblocks words.
__device__ bool grid_barrier3(unsigned* bar, unsigned nblocks, unsigned& gen, uint32_t spin_limit,
                              int32_t* flags, int* s_ok) {
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  const unsigned next = gen + 1u;
  unsigned* arrive = bar + 256;
  if (threadIdx.x == 0)
    __hip_atomic_store(&arrive[blockIdx.x], next, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  int ok = 1;
  if (blockIdx.x == 0 && threadIdx.x < 64) {
    uint32_t spins = 0;
    for (;;) {
      bool mine = true;
      for (unsigned b = threadIdx.x; b < nblocks; b += 64)
        mine = mine && (int)(__hip_atomic_load(&arrive[b], __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT) - next) >= 0;
      if (__ballot(!mine) == 0ull) break;  // uniform over the wavefront
      if (++spins > spin_limit) {
        ok = 0;
        if (threadIdx.x == 0)
          __hip_atomic_fetch_or(&flags[1], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (ok && threadIdx.x < 8)
      __hip_atomic_store(&bar[32 * threadIdx.x], next, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (threadIdx.x == 0) {
    const unsigned* rel = bar + 32 * (blockIdx.x & 7u);
    uint32_t spins = 0;
    while (ok && (int)(__hip_atomic_load(rel, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) - next) <
                     0) {
      if (++spins > spin_limit) {
        ok = 0;
        __hip_atomic_fetch_or(&flags[1], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (__hip_atomic_load(&flags[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) ok = 0;
    *s_ok = ok;
  }
  gen = next;
  __syncthreads();
  return *s_ok != 0;
}

}  // namespace hhk
