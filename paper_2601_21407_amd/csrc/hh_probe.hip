// hh_probe.hip -- issue-rate probe for the roofline denominators.
//
// Each lane runs 8 independent dependency chains of one instruction kind for
// `iters` iterations; with enough wavefronts per SIMD the chains expose the
// instruction's issue rate, not its latency.  Every chain keeps its value in
// a bounded range (2^-x, 1/x, sqrt|x|, sin of revolutions), so the probe
// never produces NaN/Inf.  The result is stored so the work is not removed.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/hh_probe.h"

namespace {

template <int OP>
__global__ __launch_bounds__(256) void k_probe(float* __restrict__ out, int iters, int n_out) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  float x[8], y[8];
  uint32_t u[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    x[c] = 0.5f + 0.01f * (float)((gid + c) & 15);
    y[c] = x[c];
    u[c] = 0x9E3779B9u * (uint32_t)(gid + c + 1);
  }
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      if (OP == HH_PROBE_FMA) x[c] = fmaf(x[c], 0.999f, 0.0001f);
      if (OP == HH_PROBE_EXP2) x[c] = __builtin_amdgcn_exp2f(-x[c]);
      if (OP == HH_PROBE_RCP) x[c] = __builtin_amdgcn_rcpf(x[c]);
      if (OP == HH_PROBE_SQRT) x[c] = __builtin_amdgcn_sqrtf(x[c]);
      if (OP == HH_PROBE_SIN) x[c] = __builtin_amdgcn_sinf(x[c]);
      if (OP == HH_PROBE_MIX) {  // one exp chain and one fma chain per slot
        x[c] = __builtin_amdgcn_exp2f(-x[c]);
        y[c] = fmaf(y[c], 0.999f, 0.0001f);
      }
      if (OP == HH_PROBE_MUL64) {
        const uint64_t p = (uint64_t)0xD2511F53u * u[c];
        u[c] = (uint32_t)p ^ (uint32_t)(p >> 32);
      }
    }
  }
  float s = 0.0f;
#pragma unroll
  for (int c = 0; c < 8; ++c) s += x[c] + y[c] + (float)(u[c] & 1u);
  if (gid < n_out) out[gid] = s;
}

}  // namespace

extern "C" int32_t hh_probe_issue(int32_t op, int32_t iters, int32_t blocks, float* out,
                                  int32_t n_out, void* stream) {
  if (iters < 1 || blocks < 1 || !out || n_out < 1) return -1;
  hipStream_t s = (hipStream_t)stream;
  const dim3 g((unsigned)blocks), b(256);
  switch (op) {
    case HH_PROBE_FMA: hipLaunchKernelGGL(k_probe<HH_PROBE_FMA>, g, b, 0, s, out, iters, n_out); break;
    case HH_PROBE_EXP2: hipLaunchKernelGGL(k_probe<HH_PROBE_EXP2>, g, b, 0, s, out, iters, n_out); break;
    case HH_PROBE_RCP: hipLaunchKernelGGL(k_probe<HH_PROBE_RCP>, g, b, 0, s, out, iters, n_out); break;
    case HH_PROBE_SQRT: hipLaunchKernelGGL(k_probe<HH_PROBE_SQRT>, g, b, 0, s, out, iters, n_out); break;
    case HH_PROBE_SIN: hipLaunchKernelGGL(k_probe<HH_PROBE_SIN>, g, b, 0, s, out, iters, n_out); break;
    case HH_PROBE_MUL64: hipLaunchKernelGGL(k_probe<HH_PROBE_MUL64>, g, b, 0, s, out, iters, n_out); break;
    case HH_PROBE_MIX: hipLaunchKernelGGL(k_probe<HH_PROBE_MIX>, g, b, 0, s, out, iters, n_out); break;
    default: return -1;
  }
  return hipGetLastError() == hipSuccess ? 0 : -3;
}
