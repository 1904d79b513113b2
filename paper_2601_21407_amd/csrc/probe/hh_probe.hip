// hh_probe.hip -- issue-rate probe for the roofline denominators.
//
// Each lane runs 8 independent dependency chains of one instruction kind for
// `iters` iterations; with enough wavefronts per SIMD the chains expose the
// instruction's issue rate, not its latency.  Every chain keeps its value in
// a bounded range (2^-x, 1/x, sqrt|x|, sin of revolutions), so the probe
// never produces NaN/Inf.  The result is stored so the work is not removed.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../../include/hh_probe.h"

namespace {

typedef _Float16 h2 __attribute__((ext_vector_type(2)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef float f16x_acc __attribute__((ext_vector_type(16)));

template <int OP>
__global__ __launch_bounds__(256) void k_probe(float* __restrict__ out, int iters, int n_out) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  if (OP == HH_PROBE_MFMA16 || OP == HH_PROBE_MFMA16_VALU) {
    // two independent accumulator chains of 32x32x16 f16 products; the
    // VALU variant adds 8 chains of 4 FMAs per product pair
    h8 a, b;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      a[j] = (_Float16)(0.01f * (float)((gid + j) & 7));
      b[j] = (_Float16)0.01f;
    }
    f16x_acc c0 = {}, c1 = {};
    float x[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) x[c] = 0.5f + 0.01f * (float)((gid + c) & 15);
    for (int it = 0; it < iters; ++it) {
      c0 = __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c0, 0, 0, 0);
      c1 = __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c1, 0, 0, 0);
      if (OP == HH_PROBE_MFMA16_VALU) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int c = 0; c < 8; ++c) x[c] = fmaf(x[c], 0.999f, 0.0001f);
      }
    }
    float s = 0.0f;
#pragma unroll
    for (int r = 0; r < 16; ++r) s += c0[r] + c1[r];
#pragma unroll
    for (int c = 0; c < 8; ++c) s += x[c];
    if (gid < n_out) out[gid] = s;
    return;
  }
  if (OP == HH_PROBE_PKFMA16) {
    h2 x[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      x[c][0] = (_Float16)(0.5f + 0.01f * (float)((gid + c) & 15));
      x[c][1] = (_Float16)(0.25f + 0.01f * (float)((gid + c) & 7));
    }
    const h2 m = {(_Float16)0.999f, (_Float16)0.998f}, k = {(_Float16)0.0001f, (_Float16)0.0002f};
    for (int it = 0; it < iters; ++it) {
#pragma unroll
      for (int c = 0; c < 8; ++c) x[c] = __builtin_elementwise_fma(x[c], m, k);
    }
    float s = 0.0f;
#pragma unroll
    for (int c = 0; c < 8; ++c) s += (float)x[c][0] + (float)x[c][1];
    if (gid < n_out) out[gid] = s;
    return;
  }
  if (OP == HH_PROBE_EXP16) {
    _Float16 x[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) x[c] = (_Float16)(0.5f + 0.01f * (float)((gid + c) & 15));
    for (int it = 0; it < iters; ++it) {
#pragma unroll
      for (int c = 0; c < 8; ++c) x[c] = __builtin_elementwise_exp2(-x[c]);
    }
    float s = 0.0f;
#pragma unroll
    for (int c = 0; c < 8; ++c) s += (float)x[c];
    if (gid < n_out) out[gid] = s;
    return;
  }
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
    case HH_PROBE_PKFMA16: hipLaunchKernelGGL(k_probe<HH_PROBE_PKFMA16>, g, b, 0, s, out, iters, n_out); break;
    case HH_PROBE_EXP16: hipLaunchKernelGGL(k_probe<HH_PROBE_EXP16>, g, b, 0, s, out, iters, n_out); break;
    case HH_PROBE_MFMA16: hipLaunchKernelGGL(k_probe<HH_PROBE_MFMA16>, g, b, 0, s, out, iters, n_out); break;
    case HH_PROBE_MFMA16_VALU:
      hipLaunchKernelGGL(k_probe<HH_PROBE_MFMA16_VALU>, g, b, 0, s, out, iters, n_out);
      break;
    default: return -1;
  }
  return hipGetLastError() == hipSuccess ? 0 : -3;
}
