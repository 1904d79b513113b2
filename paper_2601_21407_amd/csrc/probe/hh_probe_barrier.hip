// hh_probe_barrier.hip -- the barrier floor of the network time loop
// (measurement utility, built into libhh_probe, not into libhh).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../../include/hh.h"
#include "../../../include/hh_probe.h"
#include "../hh_barrier.h"

using namespace hhk;

namespace {

constexpr int kBlock = 512;  // the block size of the network kernel k_net

__global__ void k_zero_u32(unsigned* p, int count) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < count) p[j] = 0u;
}

// ---- barrier floor (measurement) -------------------------------------------
// The per-step synchronization of k_net without the neuron work: each step
// is one grid barrier, plus (mode 1) the two accumulator reads-and-clears
// per lane that follow it in k_net.  Same block size and barrier code; mode
// 2 is the flag-array barrier alone.
__global__ __launch_bounds__(kBlock) void k_barrier_floor(unsigned* bar, int32_t* flags,
                                                             unsigned long long* acc, int n,
                                                             int steps, int mode,
                                                             uint32_t spin_limit) {
  __shared__ int s_ok;
  unsigned gen = 0;
  const int i = blockIdx.x * kBlock + threadIdx.x;
  float sink = 0.0f;
  for (int t = 0; t < steps; ++t) {
    const bool ok = mode == 2 ? grid_barrier3(bar, gridDim.x, gen, spin_limit, flags, &s_ok)
                              : grid_barrier(bar, gridDim.x, gen, spin_limit, flags, &s_ok);
    if (!ok) break;
    if (mode == 1 && i < n) {
      const unsigned long long* b = acc + (size_t)(t & 1) * 2 * n;
      sink += (float)atomicExch((unsigned long long*)&b[i], 0ull);
      sink += (float)atomicExch((unsigned long long*)&b[n + i], 0ull);
    }
  }
  if (sink != 0.0f) flags[2] = 1;  // keeps the reads; never true (accumulators are zero)
}

// barrier bytes for every mode: the flag-array layout (256 + one word per
// block), rounded up to 256 bytes so that the flags and the 64-bit
// accumulators after it stay aligned
size_t bar_bytes(int32_t blocks) { return ((256 + (size_t)blocks) * 4 + 255) & ~(size_t)255; }

}  // namespace

extern "C" {

size_t hh_probe_barrier_bytes(int32_t blocks) {
  if (blocks < 1) return 0;
  return bar_bytes(blocks) + 256 + (size_t)4 * blocks * kBlock * sizeof(unsigned long long);
}

int32_t hh_probe_barrier(int32_t steps, int32_t blocks, int32_t mode, void* work,
                         size_t work_bytes, void* stream) {
  if (steps < 1 || blocks < 1 || mode < 0 || mode > 2 || !work) return HH_E_INVALID;
  if (work_bytes < hh_probe_barrier_bytes(blocks)) return HH_E_SHAPE;
  int dev = 0, ncu = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_barrier_floor, kBlock, 0) !=
          hipSuccess)
    return HH_E_HIP;
  if (blocks > ncu * per_cu) return HH_E_UNSUPPORTED;
  hipStream_t s = (hipStream_t)stream;
  unsigned* bar = (unsigned*)work;
  int32_t* flags = (int32_t*)((char*)work + bar_bytes(blocks));
  unsigned long long* acc = (unsigned long long*)((char*)work + bar_bytes(blocks) + 256);
  if ((uintptr_t)work % 256 != 0) return HH_E_INVALID;  // the 64-bit atomics need alignment
  const int n = blocks * kBlock;
  const int words = (int)(hh_probe_barrier_bytes(blocks) / 4);
  hipLaunchKernelGGL(k_zero_u32, dim3((unsigned)((words + 255) / 256)), dim3(256), 0, s,
                     (unsigned*)work, words);
  uint32_t spin = 1u << 24;
  void* args[] = {(void*)&bar, (void*)&flags, (void*)&acc, (void*)&n, (void*)&steps, (void*)&mode,
                  (void*)&spin};
  if (hipLaunchCooperativeKernel((const void*)k_barrier_floor, dim3((unsigned)blocks),
                                 dim3(kBlock), args, 0, s) != hipSuccess)
    return HH_E_HIP;
  return hipGetLastError() == hipSuccess ? HH_OK : HH_E_HIP;
}

}  // extern "C"
