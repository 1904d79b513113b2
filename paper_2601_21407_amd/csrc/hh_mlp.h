// hh_mlp.h -- layout of the surrogate MLP (7 -> 64 -> 64 -> 6) shared by
// the training, packing, inference and deployment kernels.
#pragma once
#include <stdint.h>

constexpr int MLP_IN = 7, MLP_H = 64, MLP_OUT = 6;
// hidden-layer activations (values match HH_ACT_* of hh.h)
enum { MLP_ACT_SILU = 0, MLP_ACT_HSWISH = 1 };
// packed FP32 parameter vector: W1 [7][64], b1 [64], W2 [64][64], b2 [64],
// W3 [64][6], b3 [6]  (W[k][j]: input k -> output j)
constexpr int MLP_OFF_W1 = 0;
constexpr int MLP_OFF_B1 = MLP_OFF_W1 + MLP_IN * MLP_H;
constexpr int MLP_OFF_W2 = MLP_OFF_B1 + MLP_H;
constexpr int MLP_OFF_B2 = MLP_OFF_W2 + MLP_H * MLP_H;
constexpr int MLP_OFF_W3 = MLP_OFF_B2 + MLP_H;
constexpr int MLP_OFF_B3 = MLP_OFF_W3 + MLP_H * MLP_OUT;
constexpr int MLP_NPARAM = MLP_OFF_B3 + MLP_OUT;  // 5062

// Weights as per-lane MFMA fragments (bf16) plus normalization constants.
// w1[rt][lane][j]: layer-1 A operand, row tile rt, K slot 8*(lane/32)+j
//                  (slots 0-6 x high parts, 7 bias, 8-14 x low parts, 15 zero)
// w2[ot][kb][lane][j], w3[kb][lane][j]: A operands with the hidden units of
//                  K block kb in accumulator order
// b2[ot][half][r], b3[half][r]: biases in accumulator layout
struct __attribute__((aligned(16))) MlpPacked {
  uint16_t w1[2][64][8];
  uint16_t w2[2][4][64][8];
  uint16_t w3[4][64][8];
  float b2[2][2][16];
  float b3[2][4];
  float mu_x[8], isig_x[8];  // input normalization
  float mu_y[8], sig_y[8];   // output de-normalization
};

