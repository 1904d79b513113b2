// hh_mlp.hip -- the learned k-step surrogate: a 7 -> 64 -> 64 -> 6 MLP with
// SiLU or hard-swish activations that maps (V, m, h, n, p, q, mean input
// current) to the state change over k steps, and the kernels that form its
// training set from plain trajectories.
//
// Training kernels (hh_mlp_grad) run one sample per lane-group on the VALU
// in FP32 with the weights staged in LDS; with `quantize` they round weights
// and hidden activations to bf16 exactly where the MFMA inference does, so
// the trained network is the one that is deployed.  Per-block partial
// gradients are summed in a fixed order.
//
// Inference (mlp_infer_wave) is register resident on MFMA.  Activations are
// kept transposed (hidden x sample, 32 samples per tile): the accumulator of
// v_mfma_f32_32x32x16_bf16 puts hidden unit 8(r/4) + 4(l/32) + r%4 of sample
// l%32 in register r of lane l, and eight consecutive registers of a lane
// are exactly the eight K values that lane supplies as the B operand of the
// next layer -- provided the next layer's weight fragments list the hidden
// units in that same order.  hh_mlp_pack writes the fragments in that order,
// so no activation ever goes through LDS.  The input enters as a bf16
// high/low split in the 16 K slots of the first layer, with the first-layer
// bias in the spare slot.
#include <string.h>

#include "hh_internal.h"
#include "hh_mlp.h"

using namespace hhk;

namespace {

__device__ __forceinline__ float bf16r(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return __uint_as_float(u & 0xFFFF0000u);
}
__device__ __forceinline__ uint16_t bf16bits(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float sigm(float a) { return 1.0f / (1.0f + expf(-a)); }
// hard-swish a clamp(a / 6 + 1/2, 0, 1) (Howard et al., 2019): the
// piecewise-quadratic form of SiLU, with no transcendental function
__device__ __forceinline__ float hswish_gate(float a) {
  return __builtin_amdgcn_fmed3f(fmaf(a, 1.0f / 6.0f, 0.5f), 0.0f, 1.0f);
}
// activation value (training and VALU forward) and its derivative
template <int ACT>
__device__ __forceinline__ float act_acc(float a) {
  if constexpr (ACT == MLP_ACT_HSWISH) return a * hswish_gate(a);
  return a * sigm(a);
}
template <int ACT>
__device__ __forceinline__ float dact(float a) {
  if constexpr (ACT == MLP_ACT_HSWISH) {
    // d/da a c(a), c the clamped gate: c + a / 6 inside (-3, 3)
    return a <= -3.0f ? 0.0f : (a >= 3.0f ? 1.0f : fmaf(a, 1.0f / 3.0f, 0.5f));
  }
  const float s = sigm(a);
  return s * (1.0f + a * (1.0f - s));
}

constexpr int CH = 64;  // samples per chunk in the training kernel
constexpr int LD = MLP_H + 1;

// parameters the MFMA inference holds as bf16: W1, b1 (it rides in a K slot
// of the first layer), W2 and W3; b2 and b3 initialize the FP32 accumulators
__device__ __forceinline__ bool is_bf16_param(int j) {
  return j < MLP_OFF_B2 || (j >= MLP_OFF_W3 && j < MLP_OFF_B3);
}

// Normalized network input and target of a raw sample: (x - mean) / std per
// feature, as (x - mean) * (1 / std) with 1 / std rounded once (the form the
// deployed inference uses).  norm: input mean [0..6], std [8..14], output
// mean [16..21], std [24..29].
__device__ __forceinline__ float norm_in(const float* __restrict__ nm, int i, float x) {
  return (x - nm[i]) * (1.0f / nm[8 + i]);
}
__device__ __forceinline__ float norm_out(const float* __restrict__ nm, int o, float y) {
  return (y - nm[16 + o]) * (1.0f / nm[24 + o]);
}

// Forward + backward over a range of samples; per-block partial gradients.
template <int ACT>
__global__ __launch_bounds__(256) void k_mlp_grad(const float* __restrict__ P,
                                                  const float* __restrict__ nm,
                                                  const float* __restrict__ X,
                                                  const float* __restrict__ Y, int S, int per_block,
                                                  int quant, float* __restrict__ part,
                                                  float* __restrict__ loss_part) {
  __shared__ float w[MLP_NPARAM];
  __shared__ float xs[CH][8];
  __shared__ float a1[CH][LD], h1[CH][LD], a2[CH][LD], h2[CH][LD];
  __shared__ float dy[CH][8];
  const int tid = threadIdx.x;
  for (int j = tid; j < MLP_NPARAM; j += 256) {
    const float v = P[j];
    w[j] = (quant && is_bf16_param(j)) ? bf16r(v) : v;
  }
  const float* W1 = w + MLP_OFF_W1;
  const float* B1 = w + MLP_OFF_B1;
  const float* W2 = w + MLP_OFF_W2;
  const float* B2 = w + MLP_OFF_B2;
  const float* W3 = w + MLP_OFF_W3;
  const float* B3 = w + MLP_OFF_B3;
  float g2[16], g1[2], g3[2], gb = 0.0f, lsum = 0.0f;
#pragma unroll
  for (int q = 0; q < 16; ++q) g2[q] = 0.0f;
  g1[0] = g1[1] = g3[0] = g3[1] = 0.0f;
  const float scale = 2.0f / (float)S;
  const int beg = blockIdx.x * per_block, end = min(S, beg + per_block);
  __syncthreads();
  for (int c0 = beg; c0 < end; c0 += CH) {
    const int nc = min(CH, end - c0);
    for (int e = tid; e < CH * 8; e += 256) {
      const int s = e >> 3, i = e & 7;
      float v = 0.0f, t = 0.0f;
      if (s < nc && i < MLP_IN) {
        v = norm_in(nm, i, X[(int64_t)(c0 + s) * MLP_IN + i]);
        if (quant) {  // the inference feeds x as bf16 high + low parts
          const float hi = bf16r(v);
          v = hi + bf16r(v - hi);
        }
      }
      if (s < nc && i < MLP_OUT) t = norm_out(nm, i, Y[(int64_t)(c0 + s) * MLP_OUT + i]);
      xs[s][i] = v;
      dy[s][i] = t;  // targets for now
    }
    __syncthreads();
    for (int e = tid; e < CH * MLP_H; e += 256) {
      const int s = e / MLP_H, j = e % MLP_H;
      float a = B1[j];
#pragma unroll
      for (int i = 0; i < MLP_IN; ++i) a = fmaf(W1[i * MLP_H + j], xs[s][i], a);
      const float h = act_acc<ACT>(a);
      a1[s][j] = a;
      h1[s][j] = quant ? bf16r(h) : h;
    }
    __syncthreads();
    for (int e = tid; e < CH * MLP_H; e += 256) {
      const int s = e / MLP_H, j = e % MLP_H;
      float a = B2[j];
#pragma unroll 16
      for (int k = 0; k < MLP_H; ++k) a = fmaf(W2[k * MLP_H + j], h1[s][k], a);
      const float h = act_acc<ACT>(a);
      a2[s][j] = a;
      h2[s][j] = quant ? bf16r(h) : h;
    }
    __syncthreads();
    float dyv[2] = {0.0f, 0.0f};
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int e = tid + 256 * q;
      if (e < CH * MLP_OUT) {
        const int ys = e / MLP_OUT, yo = e % MLP_OUT;
        float y = B3[yo];
#pragma unroll 16
        for (int k = 0; k < MLP_H; ++k) y = fmaf(W3[k * MLP_OUT + yo], h2[ys][k], y);
        if (ys < nc) {
          const float d = y - dy[ys][yo];
          lsum = fmaf(d, d, lsum);
          dyv[q] = d * scale;
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int e = tid + 256 * q;
      if (e < CH * MLP_OUT) dy[e / MLP_OUT][e % MLP_OUT] = dyv[q];
    }
    __syncthreads();
    // layer 3 gradients and dA2
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int e = tid + 256 * q;
      if (e < MLP_H * MLP_OUT) {
        const int k = e / MLP_OUT, o = e % MLP_OUT;
        float s = 0.0f;
#pragma unroll 4
        for (int ss = 0; ss < CH; ++ss) s = fmaf(h2[ss][k], dy[ss][o], s);
        g3[q] += s;
      }
    }
    if (tid >= 128 && tid < 128 + MLP_OUT) {
      float s = 0.0f;
      for (int ss = 0; ss < CH; ++ss) s += dy[ss][tid - 128];
      gb += s;
    }
    for (int e = tid; e < CH * MLP_H; e += 256) {
      const int s = e / MLP_H, j = e % MLP_H;
      float d = 0.0f;
#pragma unroll
      for (int o = 0; o < MLP_OUT; ++o) d = fmaf(W3[j * MLP_OUT + o], dy[s][o], d);
      a2[s][j] = d * dact<ACT>(a2[s][j]);  // dA2
    }
    __syncthreads();
    // layer 2 gradients and dA1
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int e = tid + 256 * q;
      const int k = e / MLP_H, j = e % MLP_H;
      float s = 0.0f;
#pragma unroll 4
      for (int ss = 0; ss < CH; ++ss) s = fmaf(h1[ss][k], a2[ss][j], s);
      g2[q] += s;
    }
    if (tid >= 64 && tid < 128) {
      float s = 0.0f;
      for (int ss = 0; ss < CH; ++ss) s += a2[ss][tid - 64];
      gb += s;
    }
    for (int e = tid; e < CH * MLP_H; e += 256) {
      const int s = e / MLP_H, k = e % MLP_H;
      float d = 0.0f;
#pragma unroll 16
      for (int j = 0; j < MLP_H; ++j) d = fmaf(W2[k * MLP_H + j], a2[s][j], d);
      a1[s][k] = d * dact<ACT>(a1[s][k]);  // dA1
    }
    __syncthreads();
    // layer 1 gradients
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int e = tid + 256 * q;
      if (e < MLP_IN * MLP_H) {
        const int i = e / MLP_H, j = e % MLP_H;
        float s = 0.0f;
#pragma unroll 4
        for (int ss = 0; ss < CH; ++ss) s = fmaf(xs[ss][i], a1[ss][j], s);
        g1[q] += s;
      }
    }
    if (tid < 64) {
      float s = 0.0f;
      for (int ss = 0; ss < CH; ++ss) s += a1[ss][tid];
      gb += s;
    }
    __syncthreads();
  }
  float* out = part + (int64_t)blockIdx.x * MLP_NPARAM;
#pragma unroll
  for (int q = 0; q < 16; ++q) out[MLP_OFF_W2 + tid + 256 * q] = g2[q];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int e = tid + 256 * q;
    if (e < MLP_IN * MLP_H) out[MLP_OFF_W1 + e] = g1[q];
    if (e < MLP_H * MLP_OUT) out[MLP_OFF_W3 + e] = g3[q];
  }
  if (tid < 64) out[MLP_OFF_B1 + tid] = gb;
  else if (tid < 128) out[MLP_OFF_B2 + tid - 64] = gb;
  else if (tid < 128 + MLP_OUT) out[MLP_OFF_B3 + tid - 128] = gb;
  // per-block loss: lanes' partial sums in a fixed order
  __shared__ float lred[256];
  lred[tid] = lsum;
  __syncthreads();
  if (tid == 0) {
    float s = 0.0f;
    for (int q = 0; q < 256; ++q) s += lred[q];
    loss_part[blockIdx.x] = s;
  }
}

// Sum of the per-block partial gradients (and losses): a block owns 64
// entries; its 16 lane groups each add a sixteenth of the partials, and the
// group sums are added in group order (deterministic).
constexpr int RD_J = 64, RD_G = 16;

__global__ __launch_bounds__(RD_J * RD_G) void k_mlp_reduce(const float* __restrict__ part,
                                                          const float* __restrict__ loss_part,
                                                          int nblocks, float invS,
                                                          float* __restrict__ grad,
                                                          float* __restrict__ loss) {
  __shared__ float red[RD_G][RD_J];
  const int jx = threadIdx.x % RD_J, g = threadIdx.x / RD_J;
  const int j = blockIdx.x * RD_J + jx;  // MLP_NPARAM = the loss
  const int per = (nblocks + RD_G - 1) / RD_G;
  const int b0 = g * per, b1 = min(nblocks, b0 + per);
  float s = 0.0f;
  if (j < MLP_NPARAM) {
    for (int b = b0; b < b1; ++b) s += part[(int64_t)b * MLP_NPARAM + j];
  } else if (j == MLP_NPARAM) {
    for (int b = b0; b < b1; ++b) s += loss_part[b];
  }
  red[g][jx] = s;
  __syncthreads();
  if (g == 0 && j <= MLP_NPARAM) {
    float t = 0.0f;
    for (int q = 0; q < RD_G; ++q) t += red[q][jx];
    if (j < MLP_NPARAM) grad[j] = t;
    else if (loss) *loss = t * invS;
  }
}

// Plain FP32 forward, one sample per lane (evaluation): raw inputs in,
// de-normalized outputs (state change) out.
template <int ACT>
__global__ __launch_bounds__(256) void k_mlp_fwd(const float* __restrict__ P,
                                                 const float* __restrict__ nm,
                                                 const float* __restrict__ X, int S, int quant,
                                                 float* __restrict__ Yo) {
  __shared__ float w[MLP_NPARAM];
  for (int j = threadIdx.x; j < MLP_NPARAM; j += blockDim.x) {
    const float v = P[j];
    w[j] = (quant && is_bf16_param(j)) ? bf16r(v) : v;
  }
  __syncthreads();
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  float x[MLP_IN], h[MLP_H], y[MLP_OUT];
#pragma unroll
  for (int i = 0; i < MLP_IN; ++i) {
    float v = norm_in(nm, i, X[(int64_t)s * MLP_IN + i]);
    if (quant) {
      const float hi = bf16r(v);
      v = hi + bf16r(v - hi);
    }
    x[i] = v;
  }
#pragma unroll
  for (int j = 0; j < MLP_H; ++j) {
    float a = w[MLP_OFF_B1 + j];
#pragma unroll
    for (int i = 0; i < MLP_IN; ++i) a = fmaf(w[MLP_OFF_W1 + i * MLP_H + j], x[i], a);
    h[j] = quant ? bf16r(act_acc<ACT>(a)) : act_acc<ACT>(a);
  }
#pragma unroll
  for (int o = 0; o < MLP_OUT; ++o) y[o] = w[MLP_OFF_B3 + o];
#pragma unroll 1
  for (int j = 0; j < MLP_H; ++j) {
    float a = w[MLP_OFF_B2 + j];
#pragma unroll
    for (int k = 0; k < MLP_H; ++k) a = fmaf(w[MLP_OFF_W2 + k * MLP_H + j], h[k], a);
    const float h2 = quant ? bf16r(act_acc<ACT>(a)) : act_acc<ACT>(a);
#pragma unroll
    for (int o = 0; o < MLP_OUT; ++o) y[o] = fmaf(w[MLP_OFF_W3 + j * MLP_OUT + o], h2, y[o]);
  }
#pragma unroll
  for (int o = 0; o < MLP_OUT; ++o) Yo[(int64_t)s * MLP_OUT + o] = fmaf(y[o], nm[24 + o], nm[16 + o]);
}

// ---------------------------------------------------------------------------
// packing into MFMA fragments (see the header comment)
// ---------------------------------------------------------------------------
// hidden unit that k-slot j of lane half hf holds in k-block kb
__host__ __device__ __forceinline__ int hid_of(int kb, int hf, int j) {
  return 32 * (kb >> 1) + 16 * (kb & 1) + 8 * (j >> 2) + 4 * hf + (j & 3);
}

__global__ void k_mlp_pack(const float* __restrict__ P, const float* __restrict__ norm,
                           MlpPacked* __restrict__ out) {
  const int l = threadIdx.x;  // 64 lanes
  const int hf = l >> 5, c = l & 31;
  for (int rt = 0; rt < 2; ++rt)
    for (int j = 0; j < 8; ++j) {
      const int k = 8 * hf + j;  // input slot: 0..6 x_hi, 7 bias, 8..14 x_lo, 15 zero
      const int hcol = 32 * rt + c;
      float v;
      if (k < MLP_IN) v = P[MLP_OFF_W1 + k * MLP_H + hcol];
      else if (k == 7) v = P[MLP_OFF_B1 + hcol];
      else if (k < 8 + MLP_IN) v = P[MLP_OFF_W1 + (k - 8) * MLP_H + hcol];
      else v = 0.0f;
      out->w1[rt][l][j] = bf16bits(v);
    }
  for (int ot = 0; ot < 2; ++ot)
    for (int kb = 0; kb < 4; ++kb)
      for (int j = 0; j < 8; ++j)
        out->w2[ot][kb][l][j] = bf16bits(P[MLP_OFF_W2 + hid_of(kb, hf, j) * MLP_H + 32 * ot + c]);
  for (int kb = 0; kb < 4; ++kb)
    for (int j = 0; j < 8; ++j)
      out->w3[kb][l][j] =
          bf16bits(c < MLP_OUT ? P[MLP_OFF_W3 + hid_of(kb, hf, j) * MLP_OUT + c] : 0.0f);
  if (l < 2 * 2 * 16) {  // bias of layer 2 in accumulator layout
    const int ot = l >> 5, hh = (l >> 4) & 1, r = l & 15;
    out->b2[ot][hh][r] = P[MLP_OFF_B2 + 32 * ot + 8 * (r >> 2) + 4 * hh + (r & 3)];
  }
  if (l < 8) {
    const int hh = l >> 2, r = l & 3;
    const int o = 4 * hh + r;
    out->b3[hh][r] = o < MLP_OUT ? P[MLP_OFF_B3 + o] : 0.0f;
  }
  if (l < 8) {
    out->mu_x[l] = l < MLP_IN ? norm[l] : 0.0f;
    out->isig_x[l] = l < MLP_IN ? 1.0f / norm[8 + l] : 0.0f;
    out->mu_y[l] = l < MLP_OUT ? norm[16 + l] : 0.0f;
    out->sig_y[l] = l < MLP_OUT ? norm[24 + l] : 0.0f;
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// MFMA inference of one wavefront: 64 samples, sample s owned by lane s.
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ bf16x8 frag_ld(const uint16_t* p) {
  return *reinterpret_cast<const bf16x8*>(p);
}

// two FP32 values as a bf16 pair, rounded to nearest even (one
// v_cvt_pk_bf16_f32)
__device__ __forceinline__ uint32_t pack2(float a, float b) {
  typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
  const bf2 v = {(__bf16)a, (__bf16)b};
  return __builtin_bit_cast(uint32_t, v);
}

__device__ __forceinline__ bf16x8 u4_to_frag(uint32_t a, uint32_t b, uint32_t c, uint32_t d) {
  typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
  u32x4 v = {a, b, c, d};
  return __builtin_bit_cast(bf16x8, v);
}

// Activation of an accumulator value: SiLU on v_exp_f32 + v_rcp_f32, or
// hard-swish on one clamped FMA and a multiply
template <int ACT>
__device__ __forceinline__ float act_fast(float a) {
  if constexpr (ACT == MLP_ACT_HSWISH) return a * hswish_gate(a);
  return a * rcp(1.0f + ex2(-a * kLog2e));
}

// activation of accumulator registers r0..r0+7 as a bf16 B-operand fragment
template <int ACT>
__device__ __forceinline__ bf16x8 act_frag(const f32x16& acc, int r0) {
  return u4_to_frag(pack2(act_fast<ACT>(acc[r0 + 0]), act_fast<ACT>(acc[r0 + 1])),
                    pack2(act_fast<ACT>(acc[r0 + 2]), act_fast<ACT>(acc[r0 + 3])),
                    pack2(act_fast<ACT>(acc[r0 + 4]), act_fast<ACT>(acc[r0 + 5])),
                    pack2(act_fast<ACT>(acc[r0 + 6]), act_fast<ACT>(acc[r0 + 7])));
}

// Layers 1-3 for the 32-sample tile whose layer-1 B operand is bx; returns
// the first four accumulator registers of the output tile (outputs 0-3 of
// sample l%32 in the lower half-wave, outputs 4-5 in r = 0, 1 of the upper).
template <int ACT>
__device__ __forceinline__ void mlp_tile(const MlpPacked& W, bf16x8 bx, float (&y)[4]) {
  const int l = threadIdx.x & 63;
  const int hf = l >> 5;
  const f32x16 z = {};
  const f32x16 h1a = __builtin_amdgcn_mfma_f32_32x32x16_bf16(frag_ld(&W.w1[0][l][0]), bx, z, 0, 0, 0);
  const f32x16 h1b = __builtin_amdgcn_mfma_f32_32x32x16_bf16(frag_ld(&W.w1[1][l][0]), bx, z, 0, 0, 0);
  const bf16x8 b10 = act_frag<ACT>(h1a, 0), b11 = act_frag<ACT>(h1a, 8);
  const bf16x8 b12 = act_frag<ACT>(h1b, 0), b13 = act_frag<ACT>(h1b, 8);
  // layer 2, one 32-row output tile at a time, each activated at once
  bf16x8 b2[4];
#pragma unroll
  for (int ot = 0; ot < 2; ++ot) {
    f32x16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = W.b2[ot][hf][r];
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(frag_ld(&W.w2[ot][0][l][0]), b10, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(frag_ld(&W.w2[ot][1][l][0]), b11, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(frag_ld(&W.w2[ot][2][l][0]), b12, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(frag_ld(&W.w2[ot][3][l][0]), b13, acc, 0, 0, 0);
    b2[2 * ot] = act_frag<ACT>(acc, 0);
    b2[2 * ot + 1] = act_frag<ACT>(acc, 8);
  }
  // layer 3: outputs 0..5 in the first rows of a 32-row tile
  f32x16 acc = {};
#pragma unroll
  for (int r = 0; r < 4; ++r) acc[r] = W.b3[hf][r];
#pragma unroll
  for (int kb = 0; kb < 4; ++kb)
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(frag_ld(&W.w3[kb][l][0]), b2[kb], acc, 0, 0, 0);
#pragma unroll
  for (int r = 0; r < 4; ++r) y[r] = acc[r];
}

// x[7] = raw inputs (state and mean current) of this lane's sample;
// returns dy[6] = de-normalized outputs.
template <int ACT>
__device__ __forceinline__ void mlp_infer_wave(const MlpPacked& W, const float (&x)[MLP_IN],
                                               float (&out)[MLP_OUT]) {
  const int l = threadIdx.x & 63;
  const int hf = l >> 5;
  // normalized input, split into bf16 high and low parts
  float xn[8], xl[8];
#pragma unroll
  for (int i = 0; i < MLP_IN; ++i) {
    xn[i] = (x[i] - W.mu_x[i]) * W.isig_x[i];
    xl[i] = xn[i] - bf16r(xn[i]);
  }
  xn[7] = 1.0f;  // bias slot
  xl[7] = 0.0f;
  const uint32_t hi0 = pack2(xn[0], xn[1]), hi1 = pack2(xn[2], xn[3]);
  const uint32_t hi2 = pack2(xn[4], xn[5]), hi3 = pack2(xn[6], xn[7]);
  const uint32_t lo0 = pack2(xl[0], xl[1]), lo1 = pack2(xl[2], xl[3]);
  const uint32_t lo2 = pack2(xl[4], xl[5]), lo3 = pack2(xl[6], xl[7]);
  // lanes of the lower half pass their low parts up, the upper half its high
  // parts down
  const uint32_t s0 = hf ? hi0 : lo0, s1 = hf ? hi1 : lo1, s2 = hf ? hi2 : lo2, s3 = hf ? hi3 : lo3;
  const uint32_t r0 = __shfl_xor(s0, 32), r1 = __shfl_xor(s1, 32);
  const uint32_t r2 = __shfl_xor(s2, 32), r3 = __shfl_xor(s3, 32);
  bf16x8 bx[2];
  bx[0] = hf ? u4_to_frag(r0, r1, r2, r3) : u4_to_frag(hi0, hi1, hi2, hi3);
  bx[1] = hf ? u4_to_frag(lo0, lo1, lo2, lo3) : u4_to_frag(r0, r1, r2, r3);

  // the two 32-sample tiles one after the other (fewer live registers)
  float y0[4], y1[4];
  mlp_tile<ACT>(W, bx[0], y0);
  __builtin_amdgcn_sched_barrier(0);  // keep the tiles apart: registers, not ILP, are scarce
  mlp_tile<ACT>(W, bx[1], y1);
  // gather the six outputs of sample l into lane l
  const float t0 = hf ? y0[0] : y1[0], t1 = hf ? y0[1] : y1[1];
  const float t2 = y1[2], t3 = y1[3];
  const float q0 = __shfl_xor(t0, 32), q1 = __shfl_xor(t1, 32);
  const float q2 = __shfl_xor(t2, 32), q3 = __shfl_xor(t3, 32);
  float o[MLP_OUT];
  if (!hf) {
    o[0] = y0[0]; o[1] = y0[1]; o[2] = y0[2]; o[3] = y0[3]; o[4] = q0; o[5] = q1;
  } else {
    o[0] = q0; o[1] = q1; o[2] = q2; o[3] = q3; o[4] = y1[0]; o[5] = y1[1];
  }
#pragma unroll
  for (int k = 0; k < MLP_OUT; ++k) out[k] = fmaf(o[k], W.sig_y[k], W.mu_y[k]);
}

namespace {

// MFMA inference of S samples (64 per wavefront)
template <int ACT>
__global__ __launch_bounds__(256) void k_mlp_infer(const MlpPacked* __restrict__ Wg,
                                                   const float* __restrict__ X, int S,
                                                   float* __restrict__ Yo) {
  __shared__ MlpPacked Ws;
  {
    const uint32_t* src = reinterpret_cast<const uint32_t*>(Wg);
    uint32_t* dst = reinterpret_cast<uint32_t*>(&Ws);
    for (int j = threadIdx.x; j < (int)(sizeof(MlpPacked) / 4); j += blockDim.x) dst[j] = src[j];
  }
  __syncthreads();
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  const int sc = s < S ? s : S - 1;
  float x[MLP_IN], y[MLP_OUT];
#pragma unroll
  for (int i = 0; i < MLP_IN; ++i) x[i] = X[(int64_t)sc * MLP_IN + i];
  mlp_infer_wave<ACT>(Ws, x, y);
  if (s < S)
#pragma unroll
    for (int k = 0; k < MLP_OUT; ++k) Yo[(int64_t)s * MLP_OUT + k] = y[k];
}

}  // namespace

namespace {

// ---------------------------------------------------------------------------
// training set: normalization statistics and transitions of plain trajectories
// ---------------------------------------------------------------------------
constexpr int NF = MLP_IN + MLP_OUT;  // 13 features: 7 inputs, 6 targets
constexpr int NB_NORM = 256;          // partial-sum blocks of the statistics

__device__ __forceinline__ float feature(const float* X, const float* Y, int64_t s, int f) {
  return f < MLP_IN ? X[s * MLP_IN + f] : Y[s * MLP_OUT + (f - MLP_IN)];
}

// pass 0: per-block sums of every feature; pass 1: sums of squared
// deviations from the mean (read from norm).  Binary64 accumulation, each
// block over a fixed contiguous range, lanes combined in a fixed order.
__global__ __launch_bounds__(256) void k_norm_partial(const float* __restrict__ X,
                                                      const float* __restrict__ Y, int64_t S,
                                                      int pass, const float* __restrict__ nm,
                                                      double* __restrict__ part) {
  __shared__ double red[256];
  const int64_t per = (S + NB_NORM - 1) / NB_NORM;
  const int64_t beg = blockIdx.x * per, end = beg + per < S ? beg + per : S;
  for (int f = 0; f < NF; ++f) {
    const double mu = pass ? (double)nm[f < MLP_IN ? f : 16 + f - MLP_IN] : 0.0;
    double acc = 0.0;
    for (int64_t s = beg + threadIdx.x; s < end; s += 256) {
      const double d = (double)feature(X, Y, s, f) - mu;
      acc += pass ? d * d : d;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x * NF + f] = red[0];
    __syncthreads();
  }
}

// the partial sums in block order: pass 0 writes the means, pass 1 the
// sample standard deviations (floored at 1e-6 for inputs, 1e-9 for targets)
__global__ void k_norm_final(const double* __restrict__ part, int64_t S, int pass,
                             float* __restrict__ nm) {
  const int f = threadIdx.x;
  if (f >= NF) return;
  double t = 0.0;
  for (int b = 0; b < NB_NORM; ++b) t += part[b * NF + f];
  const int slot = f < MLP_IN ? f : 16 + f - MLP_IN;
  if (pass == 0) {
    nm[slot] = (float)(t / (double)S);
  } else {
    const double sd = S > 1 ? sqrt(t / (double)(S - 1)) : 0.0;
    const double floor_ = f < MLP_IN ? 1e-6 : 1e-9;
    nm[slot + 8] = (float)(sd > floor_ ? sd : floor_);
  }
}

__global__ void k_norm_clear(float* __restrict__ nm) {
  if (threadIdx.x < 32) nm[threadIdx.x] = 0.0f;
}

// Transitions of plain trajectories.  traj [T][n_state][n] holds the state
// before every step (rows V, five gates, V_lo); step t of element i gives a
// sample when V <= v_fb before step t and before step t + k: input (state at
// t, mean input current over steps t .. t + k - 1), target (state at t + k)
// minus (state at t).  V is V + V_lo.  Samples are ordered by (t, i).
__device__ __forceinline__ bool trans_ok(const float* __restrict__ traj, int ns, int64_t n,
                                         int64_t t, int k, int64_t i, float v_fb) {
  const float va = traj[(t * ns) * n + i] + traj[(t * ns + ns - 1) * n + i];
  const float vb = traj[((t + k) * ns) * n + i] + traj[((t + k) * ns + ns - 1) * n + i];
  return va <= v_fb && vb <= v_fb;
}

// one block per step t: number of samples of step t
__global__ __launch_bounds__(256) void k_trans_count(const float* __restrict__ traj, int ns,
                                                     int64_t n, int k, float v_fb,
                                                     int64_t* __restrict__ cnt) {
  __shared__ int64_t red[4];
  const int64_t t = blockIdx.x;
  int64_t c = 0;
  for (int64_t i = threadIdx.x; i < n; i += 256) c += trans_ok(traj, ns, n, t, k, i, v_fb);
  for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) cnt[t] = (red[0] + red[1]) + (red[2] + red[3]);
}

// exclusive prefix of the per-step counts (one thread, steps in order);
// cnt[rows] receives the total
__global__ void k_trans_scan(int64_t* __restrict__ cnt, int64_t rows) {
  if (threadIdx.x != 0) return;
  int64_t run = 0;
  for (int64_t t = 0; t < rows; ++t) {
    const int64_t c = cnt[t];
    cnt[t] = run;
    run += c;
  }
  cnt[rows] = run;
}

// one block per step t: the samples of step t, in element order, from
// offset off[t]; samples at or beyond cap are dropped
__global__ __launch_bounds__(256) void k_trans_write(const float* __restrict__ traj, int ns,
                                                     int64_t n, int k, float v_fb,
                                                     const float* __restrict__ I,
                                                     const int64_t* __restrict__ off, int64_t cap,
                                                     float* __restrict__ X, float* __restrict__ Y) {
  __shared__ int wsum[4];
  const int64_t t = blockIdx.x;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int64_t base = off[t];
  for (int64_t i0 = 0; i0 < n; i0 += 256) {
    const int64_t i = i0 + threadIdx.x;
    const bool ok = i < n && trans_ok(traj, ns, n, t, k, i, v_fb);
    const uint64_t b = __ballot(ok);
    if (lane == 0) wsum[wv] = __popcll(b);
    __syncthreads();
    int before = 0;
    for (int w = 0; w < wv; ++w) before += wsum[w];
    const int tot = (wsum[0] + wsum[1]) + (wsum[2] + wsum[3]);
    if (ok) {
      const int64_t s = base + before +
          (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0u));
      if (s < cap) {
        float xa[MLP_OUT], xb[MLP_OUT];
#pragma unroll
        for (int r = 0; r < MLP_OUT; ++r) {
          xa[r] = traj[(t * ns + r) * n + i];
          xb[r] = traj[((t + k) * ns + r) * n + i];
        }
        xa[0] += traj[(t * ns + ns - 1) * n + i];
        xb[0] += traj[((t + k) * ns + ns - 1) * n + i];
        // the mean input exactly as the deployment kernel forms it
        float sum = 0.0f;
        for (int j = 0; j < k; ++j) sum += I[(t + j) * n + i];
#pragma unroll
        for (int r = 0; r < MLP_OUT; ++r) {
          X[s * MLP_IN + r] = xa[r];
          Y[s * MLP_OUT + r] = xb[r] - xa[r];
        }
        X[s * MLP_IN + MLP_OUT] = sum / (float)k;
      }
    }
    base += tot;
    __syncthreads();
  }
}

}  // namespace

extern "C" {

size_t hh_mlp_grad_workspace(int32_t S) {
  if (S < 1) return 0;
  const int nb = (S + CH - 1) / CH < 512 ? (S + CH - 1) / CH : 512;
  return (size_t)nb * (MLP_NPARAM + 1) * sizeof(float);
}

static bool act_ok(int32_t act) { return act == HH_ACT_SILU || act == HH_ACT_HARDSWISH; }

int32_t hh_mlp_grad(const float* params, const float* norm, const float* X, const float* Y,
                    int32_t S, int32_t quantize, int32_t act, float* grad, float* loss,
                    void* workspace, size_t workspace_bytes, void* stream) {
  if (!params || !norm || !X || !Y || !grad) return HH_E_INVALID;
  if (!act_ok(act)) return HH_E_INVALID;
  if (S < 1) return HH_E_SHAPE;
  if (!workspace || workspace_bytes < hh_mlp_grad_workspace(S)) return HH_E_SHAPE;
  int nb = (S + CH - 1) / CH;
  if (nb > 512) nb = 512;
  int per = (S + nb - 1) / nb;
  per = (per + CH - 1) / CH * CH;
  nb = (S + per - 1) / per;
  float* part = (float*)workspace;
  float* lpart = part + (size_t)nb * MLP_NPARAM;
  hipStream_t s = (hipStream_t)stream;
  const int q = quantize ? 1 : 0;
  if (act == HH_ACT_HARDSWISH)
    hipLaunchKernelGGL(k_mlp_grad<MLP_ACT_HSWISH>, dim3(nb), dim3(256), 0, s, params, norm, X, Y, S,
                       per, q, part, lpart);
  else
    hipLaunchKernelGGL(k_mlp_grad<MLP_ACT_SILU>, dim3(nb), dim3(256), 0, s, params, norm, X, Y, S,
                       per, q, part, lpart);
  hipLaunchKernelGGL(k_mlp_reduce, dim3((MLP_NPARAM + 1 + RD_J - 1) / RD_J), dim3(RD_J * RD_G), 0, s,
                     part, lpart, nb, 1.0f / (float)S, grad, loss);
  return hipGetLastError() == hipSuccess ? HH_OK : HH_E_HIP;
}

int32_t hh_mlp_forward(const float* params, const float* norm, const float* X, int32_t S,
                       int32_t quantize, int32_t act, float* Y, void* stream) {
  if (!params || !norm || !X || !Y) return HH_E_INVALID;
  if (!act_ok(act)) return HH_E_INVALID;
  if (S < 0) return HH_E_SHAPE;
  if (S == 0) return HH_OK;
  const dim3 g((S + 255) / 256), b(256);
  hipStream_t s = (hipStream_t)stream;
  if (act == HH_ACT_HARDSWISH)
    hipLaunchKernelGGL(k_mlp_fwd<MLP_ACT_HSWISH>, g, b, 0, s, params, norm, X, S, quantize ? 1 : 0, Y);
  else
    hipLaunchKernelGGL(k_mlp_fwd<MLP_ACT_SILU>, g, b, 0, s, params, norm, X, S, quantize ? 1 : 0, Y);
  return hipGetLastError() == hipSuccess ? HH_OK : HH_E_HIP;
}

size_t hh_mlp_norm_workspace(void) { return (size_t)NB_NORM * NF * sizeof(double); }

int32_t hh_mlp_norm(const float* X, const float* Y, int64_t S, float* norm, void* workspace,
                    size_t workspace_bytes, void* stream) {
  if (!X || !Y || !norm) return HH_E_INVALID;
  if (S < 1) return HH_E_SHAPE;
  if (!workspace || workspace_bytes < hh_mlp_norm_workspace()) return HH_E_SHAPE;
  hipStream_t s = (hipStream_t)stream;
  double* part = (double*)workspace;
  hipLaunchKernelGGL(k_norm_clear, dim3(1), dim3(64), 0, s, norm);
  for (int pass = 0; pass < 2; ++pass) {
    hipLaunchKernelGGL(k_norm_partial, dim3(NB_NORM), dim3(256), 0, s, X, Y, S, pass, norm, part);
    hipLaunchKernelGGL(k_norm_final, dim3(1), dim3(64), 0, s, part, S, pass, norm);
  }
  return hipGetLastError() == hipSuccess ? HH_OK : HH_E_HIP;
}

size_t hh_surrogate_transitions_workspace(int32_t T, int32_t k) {
  if (T < 1 || k < 1 || k >= T) return 0;
  return (size_t)(T - k + 1) * sizeof(int64_t);
}

int32_t hh_surrogate_transitions(const float* traj, int32_t n_state, const float* i_dense,
                                 int64_t n, int32_t T, int32_t k, float v_fb, float* X, float* Y,
                                 int64_t cap, int64_t* count, void* workspace,
                                 size_t workspace_bytes, void* stream) {
  if (!traj || !i_dense || !X || !Y || !count) return HH_E_INVALID;
  if (n_state != 2 + MLP_OUT - 1) return HH_E_UNSUPPORTED;  // V, five gates, V_lo
  if (n < 1 || T < 2 || k < 1 || k >= T || cap < 0) return HH_E_SHAPE;
  if (!workspace || workspace_bytes < hh_surrogate_transitions_workspace(T, k)) return HH_E_SHAPE;
  const int64_t rows = T - k;
  int64_t* cnt = (int64_t*)workspace;
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_trans_count, dim3((unsigned)rows), dim3(256), 0, s, traj, n_state, n, k, v_fb,
                     cnt);
  hipLaunchKernelGGL(k_trans_scan, dim3(1), dim3(64), 0, s, cnt, rows);
  hipLaunchKernelGGL(k_trans_write, dim3((unsigned)rows), dim3(256), 0, s, traj, n_state, n, k, v_fb,
                     i_dense, cnt, cap, X, Y);
  if (hipMemcpyAsync(count, cnt + rows, sizeof(int64_t), hipMemcpyDeviceToDevice, s) != hipSuccess)
    return HH_E_HIP;
  return hipGetLastError() == hipSuccess ? HH_OK : HH_E_HIP;
}

int32_t hh_mlp_pack(const float* params, const float* norm, void* packed, void* stream) {
  if (!params || !norm || !packed) return HH_E_INVALID;
  hipLaunchKernelGGL(k_mlp_pack, dim3(1), dim3(64), 0, (hipStream_t)stream, params, norm,
                     (MlpPacked*)packed);
  return hipGetLastError() == hipSuccess ? HH_OK : HH_E_HIP;
}

size_t hh_mlp_packed_bytes(void) { return sizeof(MlpPacked); }

int32_t hh_mlp_infer(const void* packed, int32_t act, const float* X, int32_t S, float* Y,
                     void* stream) {
  if (!packed || !X || !Y) return HH_E_INVALID;
  if (!act_ok(act)) return HH_E_INVALID;
  if (S < 0) return HH_E_SHAPE;
  if (S == 0) return HH_OK;
  const dim3 g((S + 255) / 256), b(256);
  hipStream_t s = (hipStream_t)stream;
  const MlpPacked* W = (const MlpPacked*)packed;
  if (act == HH_ACT_HARDSWISH)
    hipLaunchKernelGGL(k_mlp_infer<MLP_ACT_HSWISH>, g, b, 0, s, W, X, S, Y);
  else
    hipLaunchKernelGGL(k_mlp_infer<MLP_ACT_SILU>, g, b, 0, s, W, X, S, Y);
  return hipGetLastError() == hipSuccess ? HH_OK : HH_E_HIP;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Deployment: the surrogate advances subthreshold neurons by k steps per
// call; the plain integrator (same code as hh_step_n) takes over for a
// neuron whose V is above v_fb before or after the call, for neurons that
// failed the last periodic check, and for every neuron on check calls (every
// check_every-th call), where |V_plain - V_surrogate| > check_tol marks the
// neuron plain until the next check.  Spikes come from plain steps only.
//
// A block of SB neurons is the compaction pool: neurons that need the plain
// integrator on a call are packed into the first slots of an LDS pool, so
// the plain work runs on dense wavefronts.  Blocks are small (4 wavefronts)
// and several share a CU, so one block's plain phase overlaps the others'
// MLP phases.  Pool slots, the pool counter and the spike words are double
// buffered by call parity: two barriers per call.
// ---------------------------------------------------------------------------
namespace {

constexpr int SB = 256;  // block size = compaction pool
constexpr int KMAX = 32;  // steps per surrogate call (k * SB/32 <= SB threads clear the spike words)
constexpr int SBW = SB / 32;  // spike words per block and step
constexpr int kSBW = SB / 64;  // wavefronts per block
// Dense input of the next call prefetched into registers for calls of up to
// KPF steps (its mean is the next call's network input); longer calls load
// it when they need it.
constexpr int KPF = 16;

struct SurArgs {
  float* state;
  uint8_t* flags;
  int64_t n;
  int64_t t0;
  int32_t ncalls, k;
  int32_t in_mode;
  float mu, sigma;
  uint64_t seed;
  const float* i_dense;
  float v_fb, check_tol;
  int32_t check_every;
  uint32_t* spikes;
  int64_t words;
  unsigned long long* stats;
  const MlpPacked* W;
};

// mean input current of neuron nid over the k steps from tc (dense input:
// column col of the rows of call `call`); noise as in hh_step_n
__device__ __forceinline__ float call_mean_input(const SurArgs& A, uint32_t nid, int64_t col,
                                                 int64_t tc, int call) {
  float sum = 0.0f;
  if (A.in_mode == IN_NOISE) {
    float z[4] = {0.f, 0.f, 0.f, 0.f};
    if (tc & 3) {
      normals4(A.seed, nid, (uint64_t)tc >> 2, z);
      for (int s = 0; s < (int)(tc & 3); ++s) {
        z[0] = z[1]; z[1] = z[2]; z[2] = z[3];
      }
    }
    for (int j = 0; j < A.k; ++j) {
      const int64_t t = tc + j;
      if ((t & 3) == 0) normals4(A.seed, nid, (uint64_t)t >> 2, z);
      sum += fmaf(A.sigma, z[0], A.mu);
      z[0] = z[1]; z[1] = z[2]; z[2] = z[3];
    }
  } else if (A.in_mode == IN_DENSE) {
    const float* src = A.i_dense + (int64_t)call * A.k * A.n + col;
    for (int j = 0; j < A.k; ++j) sum += src[(int64_t)j * A.n];
  }
  return sum / (float)A.k;
}

template <class S, int ACT, int IN>
__global__ __launch_bounds__(SB, 4) void k_surrogate(KModel M, SurArgs A) {
  constexpr int NG = S::kNG;
  __shared__ MlpPacked Ws;
  __shared__ float sv[2][SB], svl[2][SB], sp[2][NG][SB];
  __shared__ int sid[2][SB];
  __shared__ uint32_t sbits[KMAX][SBW];
  __shared__ int s_cnt[2];
  {
    const uint32_t* src = reinterpret_cast<const uint32_t*>(A.W);
    uint32_t* dst = reinterpret_cast<uint32_t*>(&Ws);
    for (int j = threadIdx.x; j < (int)(sizeof(MlpPacked) / 4); j += SB) dst[j] = src[j];
  }
  const int tid = threadIdx.x, lane = tid & 63;
  if (tid < KMAX * SBW) sbits[tid / SBW][tid % SBW] = 0u;
  if (tid < 2) s_cnt[tid] = 0;
  const int64_t n = A.n;
  const int64_t blk0 = blockIdx.x * (int64_t)SB;
  const int64_t i = blk0 + tid;
  const bool act = i < n;
  const int64_t ii = act ? i : n - 1;
  LaneRates<NG> L;
  load_rates<S>(M, nullptr, 0, 1, L);
  const float dtC = M.dt / M.C;
  const int64_t row_lo = (int64_t)(1 + NG) * n;
  float vh = A.state[ii], vl = A.state[row_lo + ii], p[ng1<NG>];
#pragma unroll
  for (int g = 0; g < NG; ++g) p[g] = A.state[(int64_t)(1 + g) * n + ii];
  bool forced = A.flags[ii] != 0;
  uint32_t n_mlp = 0, n_plain = 0, n_fail = 0;
  const int64_t blk_w0 = blk0 >> 5;  // first spike word of the block
  // this neuron's dense input of the coming call, loaded one call ahead so
  // the loads are in flight during the current call's work
  const bool pf = IN == IN_DENSE && A.k <= KPF;
  float pre[KPF];
  if (pf) {
#pragma unroll
    for (int j = 0; j < KPF; ++j)
      pre[j] = j < A.k ? A.i_dense[(int64_t)j * n + ii] : 0.0f;
  }
  __syncthreads();

  for (int call = 0; call < A.ncalls; ++call) {
    const int cb = call & 1;
    const int64_t tc = A.t0 + (int64_t)call * A.k;
    const bool check = A.check_every > 0 && ((call + 1) % A.check_every) == 0;
    const bool sub = act && vh <= A.v_fb;  // surrogate admissible before the call
    float pred[MLP_OUT];
    bool cand = false;
    if (__ballot(check ? act : (sub && !forced))) {
      float x[MLP_IN] = {vh + vl, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int g = 0; g < NG && g < MLP_IN - 2; ++g) x[1 + g] = p[g];
      if (pf) {
        // the same sum in step order as call_mean_input
        float sum = 0.0f;
#pragma unroll
        for (int j = 0; j < KPF; ++j)
          if (j < A.k) sum += pre[j];
        x[MLP_IN - 1] = sum / (float)A.k;
      } else {
        x[MLP_IN - 1] = call_mean_input(A, (uint32_t)ii, ii, tc, call);
      }
      float dy[MLP_OUT];
      mlp_infer_wave<ACT>(Ws, x, dy);
      pred[0] = x[0] + dy[0];
#pragma unroll
      for (int g = 0; g < MLP_OUT - 1; ++g) pred[1 + g] = fminf(fmaxf(x[1 + g] + dy[1 + g], 0.0f), 1.0f);
      cand = sub && pred[0] <= A.v_fb;  // ... and after it
    }
    if (pf && call + 1 < A.ncalls) {
      const float* nsrc = A.i_dense + (int64_t)(call + 1) * A.k * n + ii;
#pragma unroll
      for (int j = 0; j < KPF; ++j)
        if (j < A.k) pre[j] = nsrc[(int64_t)j * n];
    }
    const bool use_mlp = cand && !forced && !check;
    const bool plain = act && !use_mlp;
    int myslot = 0;
    const uint64_t b = __ballot(plain);
    if (b) {
      int base = 0;
      if (lane == 0) base = atomicAdd(&s_cnt[cb], __popcll(b));
      base = __shfl(base, 0);
      if (plain) {
        myslot = base + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32),
                                                       __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0u));
        sv[cb][myslot] = vh;
        svl[cb][myslot] = vl;
#pragma unroll
        for (int g = 0; g < NG; ++g) sp[cb][g][myslot] = p[g];
        sid[cb][myslot] = tid;
      }
    }
    __syncthreads();  // pool of this call complete
    const int cnt = s_cnt[cb];
    // Pool slot this thread integrates: slots fill whole wavefronts (64 per
    // wavefront, so the plain work runs on as few wavefronts as possible),
    // and the wavefront that takes the first 64 slots rotates with the call.
    // The waves of a block sit on different SIMDs, so the rotation spreads
    // the plain work over all of them instead of loading one SIMD with the
    // plain phase of every block.
    const int slot = ((((tid >> 6) + kSBW - (call % kSBW)) % kSBW) << 6) | lane;
    if (slot < cnt) {
      // dense plain integration of the compacted neurons
      const int loc = sid[cb][slot];
      const int64_t nid = blk0 + loc;
      float wv = sv[cb][slot], wl = svl[cb][slot], wp[ng1<NG>];
#pragma unroll
      for (int g = 0; g < NG; ++g) wp[g] = sp[cb][g][slot];
      float z[4] = {0.f, 0.f, 0.f, 0.f};
      if (IN == IN_NOISE && (tc & 3)) {
        normals4(A.seed, (uint32_t)nid, (uint64_t)tc >> 2, z);
        for (int s = 0; s < (int)(tc & 3); ++s) {
          z[0] = z[1]; z[1] = z[2]; z[2] = z[3];
        }
      }
      const float* dsrc = A.i_dense ? A.i_dense + (int64_t)call * A.k * A.n + nid : nullptr;
      // dense input two steps ahead (the rows were just read by the owning
      // lanes for the network's mean, so they come from the caches)
      float d0 = 0.0f, d1 = 0.0f;
      if (IN == IN_DENSE) {
        d0 = dsrc[0];
        if (A.k > 1) d1 = dsrc[A.n];
      }
      for (int j = 0; j < A.k; ++j) {
        float I = 0.0f;
        if (IN == IN_NOISE) {
          const int64_t t = tc + j;
          if ((t & 3) == 0) normals4(A.seed, (uint32_t)nid, (uint64_t)t >> 2, z);
          I = fmaf(A.sigma, z[0], A.mu);
          z[0] = z[1]; z[1] = z[2]; z[2] = z[3];
        } else {
          I = d0;
          d0 = d1;
          if (j + 2 < A.k) d1 = dsrc[(int64_t)(j + 2) * A.n];
        }
        const float V = wv;
        neuron_step<S>(M, L, dtC, wv, wl, wp, I, 0.0f, 0.0f);
        if (V < M.v_th && wv >= M.v_th) atomicOr(&sbits[j][loc >> 5], 1u << (loc & 31));
      }
      sv[cb][slot] = wv;
      svl[cb][slot] = wl;
#pragma unroll
      for (int g = 0; g < NG; ++g) sp[cb][g][slot] = wp[g];
    }
    if (tid == 0) s_cnt[cb ^ 1] = 0;  // counter of the next call (last read before this call)
    __syncthreads();  // plain results and spike bits complete
    if (tid < A.k * SBW) {
      // the block's spike words of this call; cleared for the next call by
      // the same thread
      const int j = tid / SBW, w = tid % SBW;
      const int64_t wd = blk_w0 + w;
      if (A.spikes && wd < A.words) A.spikes[((int64_t)call * A.k + j) * A.words + wd] = sbits[j][w];
      sbits[j][w] = 0u;
    }
    if (plain) {
      const float vp = sv[cb][myslot];
      if (check && cand) {
        const bool fail = fabsf(vp - pred[0]) > A.check_tol;
        forced = fail;
        n_fail += fail;
      }
      vh = vp;
      vl = svl[cb][myslot];
#pragma unroll
      for (int g = 0; g < NG; ++g) p[g] = sp[cb][g][myslot];
      n_plain += 1;
    } else if (use_mlp) {
      vh = pred[0];
      vl = 0.0f;
#pragma unroll
      for (int g = 0; g < NG; ++g) p[g] = pred[1 + g];
      n_mlp += 1;
    }
  }
  if (act) {
    A.state[i] = vh;
    A.state[row_lo + i] = vl;
#pragma unroll
    for (int g = 0; g < NG; ++g) A.state[(int64_t)(1 + g) * n + i] = p[g];
    A.flags[i] = forced ? 1 : 0;
  }
  if (A.stats) {
    // wave totals, one atomic per wave and counter
    uint32_t a = n_mlp, c = n_plain, f = n_fail;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      a += __shfl_xor(a, off);
      c += __shfl_xor(c, off);
      f += __shfl_xor(f, off);
    }
    if (lane == 0) {
      atomicAdd(&A.stats[0], (unsigned long long)a);
      atomicAdd(&A.stats[1], (unsigned long long)c);
      atomicAdd(&A.stats[2], (unsigned long long)f);
    }
  }
}

}  // namespace

extern "C" int32_t hh_surrogate_step_n(hh_model* m, const void* mlp_packed, int32_t act,
                                       float* state,
                                       uint8_t* flags, int64_t t0, int32_t n_steps, int32_t k,
                                       const hh_input* in, float v_fallback, int32_t check_every,
                                       float check_tol, uint32_t* spikes, uint64_t* stats,
                                       void* stream) {
  if (!m || !mlp_packed || !state || !flags || !in) return HH_E_INVALID;
  if (act != HH_ACT_SILU && act != HH_ACT_HARDSWISH) return HH_E_INVALID;
  if (k < 1 || k > KMAX || n_steps < 0 || n_steps % k != 0 || t0 < 0 || check_every < 0)
    return HH_E_SHAPE;
  if (in->mode == HH_IN_CONST || in->mode == HH_IN_BACKGROUND || in->mode == HH_IN_SINE)
    return HH_E_UNSUPPORTED;
  if (in->mode == HH_IN_DENSE && !in->i_dense) return HH_E_INVALID;
  if (m->km.has_syn || m->coef || m->cm || m->B != 1 || m->d_tab || m->d_cable)
    return HH_E_UNSUPPORTED;
  if (!CorticalSpec::matches(m->km)) return HH_E_UNSUPPORTED;
  if (n_steps == 0) return HH_OK;
  SurArgs a;
  memset(&a, 0, sizeof(a));
  a.state = state;
  a.flags = flags;
  a.n = m->n;
  a.t0 = t0;
  a.ncalls = n_steps / k;
  a.k = k;
  a.in_mode = in->mode;
  a.mu = in->mu;
  a.sigma = in->sigma;
  a.seed = in->seed;
  a.i_dense = in->i_dense;
  a.v_fb = v_fallback;
  a.check_tol = check_tol;
  a.check_every = check_every;
  a.spikes = spikes;
  a.words = (m->n + 31) / 32;
  a.stats = (unsigned long long*)stats;
  a.W = (const MlpPacked*)mlp_packed;
  const int64_t nb = (m->n + SB - 1) / SB;
  const dim3 g((unsigned)nb), b(SB);
  hipStream_t s = (hipStream_t)stream;
  const bool dense = in->mode == HH_IN_DENSE;
  if (act == HH_ACT_HARDSWISH) {
    if (dense) hipLaunchKernelGGL((k_surrogate<CorticalSpec, MLP_ACT_HSWISH, IN_DENSE>), g, b, 0, s, m->km, a);
    else hipLaunchKernelGGL((k_surrogate<CorticalSpec, MLP_ACT_HSWISH, IN_NOISE>), g, b, 0, s, m->km, a);
  } else {
    if (dense) hipLaunchKernelGGL((k_surrogate<CorticalSpec, MLP_ACT_SILU, IN_DENSE>), g, b, 0, s, m->km, a);
    else hipLaunchKernelGGL((k_surrogate<CorticalSpec, MLP_ACT_SILU, IN_NOISE>), g, b, 0, s, m->km, a);
  }
  return hipGetLastError() == hipSuccess ? HH_OK : HH_E_HIP;
}
