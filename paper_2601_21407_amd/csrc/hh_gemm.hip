// hh_gemm.hip -- dense input projection of the differentiable layer on MFMA.
//
//   forward   out[M][N] = A[M][K] . W[K][N]          (bf16 x bf16 -> fp32)
//   wgrad     dW[K][N]  = A^T . dOut                  (dOut fp32 split into
//                                                      bf16 hi + lo terms)
//
// Tiling: a 256-lane block computes a 128 x 128 output tile; its four
// wavefronts each own 64 x 64 = 2 x 2 tiles of v_mfma_f32_32x32x16_bf16.
// The block stages a 128 x 32 slab of each operand through LDS per
// iteration, laid out so that every lane reads its 8 consecutive K values
// of an MFMA operand as one 16-byte LDS read.  Rows are padded by 8 bf16
// to spread LDS banks.
//
// MFMA 32x32x16 operand layout (lane l): A row l%32, k = 8*(l/32)..+7;
// B column l%32, same k; accumulator register r holds row
// 8*(r/4) + 4*(l/32) + r%4, column l%32.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/hh.h"

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int BM = 128, BN = 128, BK = 32, LDSK = BK + 8;

__device__ __forceinline__ uint16_t f2bf(float f) {
  // round to nearest even
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ bf16x8 lds8(const uint16_t* p) {
  return *reinterpret_cast<const bf16x8*>(p);
}

// XCD-aware tile order: consecutive block ids go to different XCDs
// (round-robin over 8), so the 8 column tiles of one row panel are given to
// ids that share id % 8 -- they run on the same XCD and share its L2 copy of
// the row panel.
__device__ __forceinline__ void tile_of(int b, int tiles_m, int tiles_n, int& tm, int& tn) {
  if (tiles_n == 8 && tiles_m % 8 == 0) {
    tn = (b >> 3) & 7;
    tm = (b & 7) + 8 * (b >> 6);
  } else {
    tm = b / tiles_n;
    tn = b % tiles_n;
  }
}

__global__ __launch_bounds__(256) void k_proj_fwd(const uint16_t* __restrict__ A,
                                                  const uint16_t* __restrict__ W,
                                                  float* __restrict__ C, int M, int N, int K) {
  __shared__ __attribute__((aligned(16))) uint16_t As[BM * LDSK];  // [m][k]
  __shared__ __attribute__((aligned(16))) uint16_t Bs[BN * LDSK];  // [n][k]
  const int tiles_m = (M + BM - 1) / BM, tiles_n = (N + BN - 1) / BN;
  int tm, tn;
  tile_of(blockIdx.x, tiles_m, tiles_n, tm, tn);
  const int m0 = tm * BM, n0 = tn * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  f32x16 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;

  for (int k0 = 0; k0 < K; k0 += BK) {
    // A slab: 128 rows x 32 k, as 4-element pieces (rows are only 8-byte aligned)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int piece = tid + 256 * q;  // 0..1023
      const int r = piece >> 3, kc = (piece & 7) * 4;
      const int gm = m0 + r, gk = k0 + kc;
      uint16_t v[4] = {0, 0, 0, 0};
      if (gm < M) {
        const uint16_t* src = A + (int64_t)gm * K + gk;
        if (gk + 3 < K && ((((uintptr_t)src) & 7u) == 0)) {
          const uint2 w2 = *reinterpret_cast<const uint2*>(src);
          v[0] = (uint16_t)w2.x; v[1] = (uint16_t)(w2.x >> 16);
          v[2] = (uint16_t)w2.y; v[3] = (uint16_t)(w2.y >> 16);
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (gk + e < K) v[e] = src[e];
        }
      }
      uint16_t* dst = As + r * LDSK + kc;
#pragma unroll
      for (int e = 0; e < 4; ++e) dst[e] = v[e];
    }
    // W slab: 32 k rows x 128 n, stored transposed
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int piece = tid + 256 * q;  // 0..511
      const int kr = piece >> 4, nc = (piece & 15) * 8;
      const int gk = k0 + kr, gn = n0 + nc;
      uint16_t v[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = 0;
      if (gk < K) {
        const uint16_t* src = W + (int64_t)gk * N + gn;
        if (gn + 7 < N && ((((uintptr_t)src) & 15u) == 0)) {
          const uint4 w4 = *reinterpret_cast<const uint4*>(src);
          const uint32_t ww[4] = {w4.x, w4.y, w4.z, w4.w};
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            v[2 * e] = (uint16_t)ww[e];
            v[2 * e + 1] = (uint16_t)(ww[e] >> 16);
          }
        } else {
#pragma unroll
          for (int e = 0; e < 8; ++e)
            if (gn + e < N) v[e] = src[e];
        }
      }
#pragma unroll
      for (int e = 0; e < 8; ++e) Bs[(nc + e) * LDSK + kr] = v[e];
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK; kk += 16) {
      const int kl = kk + 8 * (lane >> 5);
      bf16x8 a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = lds8(As + (wm * 64 + i * 32 + (lane & 31)) * LDSK + kl);
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = lds8(Bs + (wn * 64 + j * 32 + (lane & 31)) * LDSK + kl);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = m0 + wm * 64 + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int col = n0 + wn * 64 + j * 32 + (lane & 31);
        if (row < M && col < N) C[(int64_t)row * N + col] = acc[i][j][r];
      }
}

// Weight gradient, one split of the reduction over M per blockIdx.y.
// Output tile: 128 (k) x 128 (n).  Per iteration 32 rows of M are staged:
// A^T slab [k][m] and dOut^T slabs [n][m] as bf16 hi and lo parts.
__global__ __launch_bounds__(256) void k_proj_wgrad(const uint16_t* __restrict__ A,
                                                    const float* __restrict__ D,
                                                    float* __restrict__ part, int M, int N, int K,
                                                    int rows_per_split) {
  __shared__ __attribute__((aligned(16))) uint16_t As[BM * LDSK];   // [k][m]
  __shared__ __attribute__((aligned(16))) uint16_t Bh[BN * LDSK];   // [n][m]
  __shared__ __attribute__((aligned(16))) uint16_t Bl[BN * LDSK];   // [n][m]
  const int tiles_k = (K + BM - 1) / BM, tiles_n = (N + BN - 1) / BN;
  const int tk = blockIdx.x / tiles_n, tn = blockIdx.x % tiles_n;
  (void)tiles_k;
  const int k0 = tk * BM, n0 = tn * BN;
  const int mbeg = blockIdx.y * rows_per_split;
  const int mend = min(M, mbeg + rows_per_split);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  f32x16 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;

  for (int ms = mbeg; ms < mend; ms += BK) {
    // A slab: 32 m rows x 128 k columns -> As[k][m]
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int piece = tid + 256 * q;  // 0..1023: 32 rows x 32 pieces of 4
      const int mr = piece >> 5, kc = (piece & 31) * 4;
      const int gm = ms + mr, gk = k0 + kc;
      uint16_t v[4] = {0, 0, 0, 0};
      if (gm < mend) {
        const uint16_t* src = A + (int64_t)gm * K + gk;
        if (gk + 3 < K && ((((uintptr_t)src) & 7u) == 0)) {
          const uint2 w2 = *reinterpret_cast<const uint2*>(src);
          v[0] = (uint16_t)w2.x; v[1] = (uint16_t)(w2.x >> 16);
          v[2] = (uint16_t)w2.y; v[3] = (uint16_t)(w2.y >> 16);
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (gk + e < K) v[e] = src[e];
        }
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) As[(kc + e) * LDSK + mr] = v[e];
    }
    // dOut slab: 32 m rows x 128 n columns (fp32) -> Bh/Bl[n][m]
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int piece = tid + 256 * q;  // 32 rows x 32 pieces of 4 floats
      const int mr = piece >> 5, nc = (piece & 31) * 4;
      const int gm = ms + mr, gn = n0 + nc;
      float v[4] = {0.f, 0.f, 0.f, 0.f};
      if (gm < mend) {
        const float* src = D + (int64_t)gm * N + gn;
        if (gn + 3 < N && ((((uintptr_t)src) & 15u) == 0)) {
          const float4 f4 = *reinterpret_cast<const float4*>(src);
          v[0] = f4.x; v[1] = f4.y; v[2] = f4.z; v[3] = f4.w;
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (gn + e < N) v[e] = src[e];
        }
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const uint16_t hi = f2bf(v[e]);
        Bh[(nc + e) * LDSK + mr] = hi;
        Bl[(nc + e) * LDSK + mr] = f2bf(v[e] - bf2f(hi));
      }
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK; kk += 16) {
      const int kl = kk + 8 * (lane >> 5);
      bf16x8 a[2], bh[2], bl[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = lds8(As + (wm * 64 + i * 32 + (lane & 31)) * LDSK + kl);
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        bh[j] = lds8(Bh + (wn * 64 + j * 32 + (lane & 31)) * LDSK + kl);
        bl[j] = lds8(Bl + (wn * 64 + j * 32 + (lane & 31)) * LDSK + kl);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], bh[j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], bl[j], acc[i][j], 0, 0, 0);
        }
    }
    __syncthreads();
  }
  float* P = part + (int64_t)blockIdx.y * K * N;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = k0 + wm * 64 + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int col = n0 + wn * 64 + j * 32 + (lane & 31);
        if (row < K && col < N) P[(int64_t)row * N + col] = acc[i][j][r];
      }
}

// Sum of the split partials in a fixed order (deterministic).
__global__ __launch_bounds__(256) void k_sum_splits(const float* __restrict__ part,
                                                    float* __restrict__ out, int64_t count,
                                                    int splits) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= count) return;
  float s = 0.0f;
  for (int q = 0; q < splits; ++q) s += part[(int64_t)q * count + i];
  out[i] = s;
}

int wgrad_splits(int M) {
  // enough blocks to fill the chip; each split reduces at least 256 rows
  int s = (M + 2047) / 2048;
  if (s > 64) s = 64;
  return s < 1 ? 1 : s;
}

}  // namespace

extern "C" {

int32_t hh_proj_forward(const uint16_t* A, const uint16_t* W, float* out, int32_t M, int32_t N,
                        int32_t K, void* stream) {
  if (!A || !W || !out) return HH_E_INVALID;
  if (M < 0 || N < 0 || K < 0) return HH_E_SHAPE;
  if (M == 0 || N == 0) return HH_OK;
  const int tiles = ((M + BM - 1) / BM) * ((N + BN - 1) / BN);
  hipLaunchKernelGGL(k_proj_fwd, dim3(tiles), dim3(256), 0, (hipStream_t)stream, A, W, out, M, N, K);
  return hipGetLastError() == hipSuccess ? HH_OK : HH_E_HIP;
}

size_t hh_proj_wgrad_workspace(int32_t M, int32_t N, int32_t K) {
  if (M <= 0 || N <= 0 || K <= 0) return 0;
  return (size_t)wgrad_splits(M) * (size_t)K * (size_t)N * sizeof(float);
}

int32_t hh_proj_wgrad(const uint16_t* A, const float* dOut, float* dW, int32_t M, int32_t N,
                      int32_t K, void* workspace, size_t workspace_bytes, void* stream) {
  if (!A || !dOut || !dW) return HH_E_INVALID;
  if (M < 0 || N < 0 || K < 0) return HH_E_SHAPE;
  if (N == 0 || K == 0) return HH_OK;
  const size_t need = hh_proj_wgrad_workspace(M > 0 ? M : 1, N, K);
  if (!workspace || workspace_bytes < need) return HH_E_SHAPE;
  const int splits = wgrad_splits(M > 0 ? M : 1);
  int rows = (M + splits - 1) / splits;
  rows = (rows + BK - 1) / BK * BK;
  const int tiles = ((K + BM - 1) / BM) * ((N + BN - 1) / BN);
  hipStream_t s = (hipStream_t)stream;
  float* part = (float*)workspace;
  hipLaunchKernelGGL(k_proj_wgrad, dim3(tiles, splits), dim3(256), 0, s, A, dOut, part, M, N, K,
                     rows);
  const int64_t count = (int64_t)K * N;
  hipLaunchKernelGGL(k_sum_splits, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, part, dW,
                     count, splits);
  return hipGetLastError() == hipSuccess ? HH_OK : HH_E_HIP;
}

}  // extern "C"
