// hh_train.hip -- the small dense pieces around the differentiable HH layer:
// linear readout of the mean spike level with cross entropy (forward and
// backward in one call) and the Adam update (Methods, "Training and
// preprocessing": Adam optimizer).  All reductions run in a fixed order, so
// results are bit-reproducible.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <mutex>

#include "../../include/hh.h"

namespace {

constexpr int kMaxC = 32;

// Butterfly sum / max over the 64 lanes of a wavefront.  Each step adds a
// lane's value and its partner's, which is the same sum in either order, so
// every lane ends with the identical, order-fixed result (deterministic).
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}
__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off));
  return v;
}

// One block per batch row: logits, softmax, per-row loss, dz = (p - y) / B
// and dL/dr for the row (r = level / T, the rate hh_backward differentiates).
// The softmax runs on the first wavefront, one class per lane.
__global__ __launch_bounds__(256) void k_readout_row(const float* __restrict__ level, float invT,
                                                     const float* __restrict__ W,
                                                     const float* __restrict__ bias,
                                                     const int32_t* __restrict__ labels, int B,
                                                     int H, int C, float* __restrict__ dz,
                                                     float* __restrict__ row_loss,
                                                     float* __restrict__ dlevel,
                                                     float* __restrict__ logits_out) {
  __shared__ float red[4][kMaxC];
  __shared__ float s_dz[kMaxC];
  const int b = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  float acc[kMaxC];
#pragma unroll
  for (int c = 0; c < kMaxC; ++c) acc[c] = 0.0f;
  for (int h = tid; h < H; h += blockDim.x) {
    const float r = level[(int64_t)b * H + h] * invT;
#pragma unroll
    for (int c = 0; c < kMaxC; ++c)
      if (c < C) acc[c] = fmaf(r, W[(int64_t)h * C + c], acc[c]);
  }
  // each wavefront's sums, then the four in order
#pragma unroll
  for (int c = 0; c < kMaxC; ++c) {
    if (c < C) {
      const float v = wave_sum(acc[c]);
      if (lane == 0) red[wv][c] = v;
    }
  }
  __syncthreads();
  if (wv == 0) {
    const bool ok = lane < C;
    const int c = ok ? lane : 0;
    const float z = ((red[0][c] + red[1][c]) + (red[2][c] + red[3][c])) + bias[c];
    const float zmax = wave_max(ok ? z : -INFINITY);
    const float ez = ok ? expf(z - zmax) : 0.0f;
    const float se = wave_sum(ez);
    const int y = labels[b];
    if (ok) {
      const float d = (ez / se - (lane == y ? 1.0f : 0.0f)) / (float)B;
      s_dz[lane] = d;
      dz[(int64_t)b * C + lane] = d;
      if (logits_out) logits_out[(int64_t)b * C + lane] = z;
      if (lane == y) row_loss[b] = -(z - zmax - logf(se));
    }
  }
  __syncthreads();
  for (int h = tid; h < H; h += blockDim.x) {
    float s = 0.0f;
    for (int c = 0; c < C; ++c) s = fmaf(s_dz[c], W[(int64_t)h * C + c], s);
    dlevel[(int64_t)b * H + h] = s;  // dL/dr, r = level / T
  }
}

// dW[h][c] = sum_b r[b][h] dz[b][c]; db[c] = sum_b dz[b][c]; loss = mean.
// Block (x, c) owns readout rows h = 32 x .. 32 x + 31 of class c; its 8
// lane groups each sum every 8th batch row, and the eight partial sums are
// added in group order.  Blocks (0, c) also form db[c], block (0, 0) the
// loss: each lane sums every 256th row, then wavefront butterflies and the
// four wavefront sums in order (all fixed orders: deterministic).
constexpr int RW_H = 32, RW_G = 8;

__global__ __launch_bounds__(RW_H * RW_G) void k_readout_wgrad(
    const float* __restrict__ level, float invT, const float* __restrict__ dz,
    const float* __restrict__ row_loss, int B, int H, int C, float* __restrict__ dW,
    float* __restrict__ db, float* __restrict__ loss) {
  __shared__ float part[RW_G][RW_H + 1];
  __shared__ float wsum[2][4];
  const int tid = threadIdx.x, hx = tid % RW_H, g = tid / RW_H;
  const int c = blockIdx.y;
  const int h = blockIdx.x * RW_H + hx;
  float acc = 0.0f;
  if (h < H) {
#pragma unroll 8
    for (int b = g; b < B; b += RW_G)
      acc = fmaf(level[(int64_t)b * H + h] * invT, dz[(int64_t)b * C + c], acc);
  }
  part[g][hx] = acc;
  if (blockIdx.x == 0) {
    float sd = 0.0f, sl = 0.0f;
    for (int b = tid; b < B; b += RW_H * RW_G) {
      sd += dz[(int64_t)b * C + c];
      if (c == 0) sl += row_loss[b];
    }
    sd = wave_sum(sd);
    sl = wave_sum(sl);
    if ((tid & 63) == 0) {
      wsum[0][tid >> 6] = sd;
      wsum[1][tid >> 6] = sl;
    }
  }
  __syncthreads();
  if (g == 0 && h < H) {
    float s = 0.0f;
    for (int q = 0; q < RW_G; ++q) s += part[q][hx];
    dW[(int64_t)h * C + c] = s;
  }
  if (blockIdx.x == 0 && tid == 0) {
    db[c] = (wsum[0][0] + wsum[0][1]) + (wsum[0][2] + wsum[0][3]);
    if (c == 0) *loss = ((wsum[1][0] + wsum[1][1]) + (wsum[1][2] + wsum[1][3])) / (float)B;
  }
}

__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v,
                                              int64_t count, float lr, float b1, float b2,
                                              float eps, float c1, float c2,
                                              uint16_t* __restrict__ p16) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= count) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float pi = p[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
  p[i] = pi;
  if (p16) {
    uint32_t u = __float_as_uint(pi);
    u += 0x7FFFu + ((u >> 16) & 1u);
    p16[i] = (uint16_t)(u >> 16);
  }
}

__global__ __launch_bounds__(256) void k_level_rate(const float* __restrict__ level, int64_t n,
                                                    float invT, float* __restrict__ rate) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) rate[i] = level[i] * invT;
}

}  // namespace

extern "C" {

int32_t hh_level_rate(const float* level, int64_t n, int32_t T, float* rate, void* stream) {
  if (!level || !rate) return HH_E_INVALID;
  if (n < 0 || T < 1) return HH_E_SHAPE;
  if (n == 0) return HH_OK;
  // the readout kernels scale the level by the same binary32 1/T
  hipLaunchKernelGGL(k_level_rate, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                     (hipStream_t)stream, level, n, 1.0f / (float)T, rate);
  return hipGetLastError() == hipSuccess ? HH_OK : HH_E_HIP;
}

size_t hh_readout_ce_workspace(int32_t B, int32_t C) {
  if (B < 1 || C < 1) return 0;
  return (size_t)B * (C + 1) * sizeof(float);
}

}  // extern "C"

// Argument checks shared by both readout entry points (scratch aside).
static int32_t readout_args_ok(const float* level, int32_t T, const float* W, const float* bias,
                               const int32_t* labels, int32_t B, int32_t H, int32_t C,
                               const float* loss, const float* dlevel, const float* dW,
                               const float* db) {
  if (!level || !W || !bias || !labels || !loss || !dlevel || !dW || !db) return HH_E_INVALID;
  if (T < 1 || B < 1 || H < 1 || C < 1) return HH_E_SHAPE;
  if (C > kMaxC) return HH_E_UNSUPPORTED;
  return HH_OK;
}

// The two readout kernels; scratch holds dz [B][C] then the row losses [B]
// (every element used is written before it is read, so nothing is cleared).
static int32_t readout_launch(const float* level, int32_t T, const float* W, const float* bias,
                              const int32_t* labels, int32_t B, int32_t H, int32_t C, float* loss,
                              float* dlevel, float* dW, float* db, float* logits, float* scratch,
                              hipStream_t s) {
  float* dz = scratch;
  float* row_loss = dz + (size_t)B * C;
  const float invT = 1.0f / (float)T;
  hipLaunchKernelGGL(k_readout_row, dim3(B), dim3(256), 0, s, level, invT, W, bias, labels, B, H, C,
                     dz, row_loss, dlevel, logits);
  hipLaunchKernelGGL(k_readout_wgrad, dim3((unsigned)((H + RW_H - 1) / RW_H), (unsigned)C),
                     dim3(RW_H * RW_G), 0, s, level, invT, dz, row_loss, B, H, C, dW, db, loss);
  return hipGetLastError() == hipSuccess ? HH_OK : HH_E_HIP;
}

// Scratch of hh_readout_ce_noalloc: a file-scope device array, one copy per
// GPU, held until the process ends.  Host code never passes the array's name
// to a kernel (on the host it is only a stand-in for the symbol): the
// device address comes from hipGetSymbolAddress, taken once per device on
// the entry point's first call there, with that device current.
static __device__ __align__(256) float scratch[HH_READOUT_NOALLOC_MAX_FLOATS];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

static int32_t scratch_of_current_device(float** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return HH_E_HIP;
  if (dev < 0 || dev >= kMaxDevices) return HH_E_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return HH_E_HIP;
    g_scratch_ptr[dev] = (float*)p;
  }
  *out = g_scratch_ptr[dev];
  return HH_OK;
}

extern "C" {

int32_t hh_readout_ce(const float* level, int32_t T, const float* W, const float* bias,
                      const int32_t* labels, int32_t B, int32_t H, int32_t C, float* loss,
                      float* dlevel, float* dW, float* db, float* logits, void* workspace,
                      size_t workspace_bytes, void* stream) {
  const int32_t st = readout_args_ok(level, T, W, bias, labels, B, H, C, loss, dlevel, dW, db);
  if (st != HH_OK) return st;
  if (!workspace || workspace_bytes < hh_readout_ce_workspace(B, C)) return HH_E_SHAPE;
  return readout_launch(level, T, W, bias, labels, B, H, C, loss, dlevel, dW, db, logits,
                        (float*)workspace, (hipStream_t)stream);
}

int32_t hh_readout_ce_noalloc(const float* level, int32_t T, const float* W, const float* bias,
                              const int32_t* labels, int32_t B, int32_t H, int32_t C, float* loss,
                              float* dlevel, float* dW, float* db, float* logits, void* stream) {
  const int32_t st = readout_args_ok(level, T, W, bias, labels, B, H, C, loss, dlevel, dW, db);
  if (st != HH_OK) return st;
  if ((int64_t)B * (C + 1) > (int64_t)HH_READOUT_NOALLOC_MAX_FLOATS) return HH_E_SHAPE;
  float* ws = nullptr;
  const int32_t sp = scratch_of_current_device(&ws);
  if (sp != HH_OK) return sp;
  return readout_launch(level, T, W, bias, labels, B, H, C, loss, dlevel, dW, db, logits, ws,
                        (hipStream_t)stream);
}

int32_t hh_adam_step(float* param, const float* grad, float* m, float* v, int64_t count, float lr,
                     float beta1, float beta2, float eps, int32_t step, uint16_t* param_bf16,
                     void* stream) {
  if (!param || !grad || !m || !v) return HH_E_INVALID;
  if (count < 0 || step < 1) return HH_E_SHAPE;
  if (!(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
    return HH_E_INVALID;
  if (count == 0) return HH_OK;
  const float c1 = (float)(1.0 / (1.0 - pow((double)beta1, (double)step)));
  const float c2 = (float)(1.0 / (1.0 - pow((double)beta2, (double)step)));
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                     param, grad, m, v, count, lr, beta1, beta2, eps, c1, c2, param_bf16);
  return hipGetLastError() == hipSuccess ? HH_OK : HH_E_HIP;
}

}  // extern "C"
