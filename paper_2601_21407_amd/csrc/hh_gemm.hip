// hh_gemm.hip -- dense input projection of the differentiable layer on MFMA.
//
//   forward   out[M][N] = A[M][K] . Wt[N][K]^T        (bf16 x bf16 -> fp32)
//   wgrad     dWt[N][K] = dOut^T . A                  (dOut fp32 split into
//                                                      bf16 hi + lo terms)
//
// The weights are kept as Wt [N][K] (K contiguous), so both operands of the
// forward product are K-contiguous rows and every lane's MFMA operand -- 8
// consecutive K values -- is one 16-byte LDS read of a row-major slab, with
// no transposition anywhere.
//
// MFMA 32x32x16 operand layout (lane l): A row l%32, k = 8*(l/32)..+7;
// B column l%32, same k; accumulator register r holds row
// 8*(r/4) + 4*(l/32) + r%4, column l%32.
//
// Forward: a 512-lane block computes a 256 x 128 output tile; its eight
// wavefronts each own 64 x 64 = 2 x 2 MFMA tiles.  Slabs of 32 K values of
// both operands are staged through two LDS buffers; the global loads of slab
// s+2 are issued (into one of two register sets) while slab s is multiplied,
// so one barrier per slab suffices.  Rows are padded to 40 bf16 (80 bytes), which makes the
// 16-byte fragment reads of eight consecutive rows hit all banks once.
//
// Weight gradient: the reduction runs over M, the slow dimension of both
// A and dOut.  A block spans all of K (up to 768 columns) for 64 columns of
// dOut, so the large fp32 operand is read once; each lane gathers eight
// consecutive rows of one dOut column (coalesced across lanes) and writes
// them as an M-contiguous LDS row.  The reduction over M is split across
// blocks and the partials are added in a fixed order.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/hh.h"

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int FBM = 256, FBN = 128, SK = 32, LDK = SK + 8;

__device__ __forceinline__ uint16_t f2bf(float f) {
  // round to nearest even
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
// two floats to a bf16 pair (round to nearest even; one conversion instruction)
__device__ __forceinline__ uint32_t pack_bf16(float a, float b) {
  typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
  const bf2 v = {(__bf16)a, (__bf16)b};
  return __builtin_bit_cast(uint32_t, v);
}

__device__ __forceinline__ bf16x8 lds8(const uint16_t* p) {
  return *reinterpret_cast<const bf16x8*>(p);
}

// XCD-aware tile order: consecutive block ids run on different XCDs (round
// robin over 8), so block b takes logical tile (b % 8) * per + b / 8: each
// XCD walks a contiguous range of row panels, and the column tiles of a
// panel share that XCD's L2 copy of it.  Returns false for the padding ids.
__device__ __forceinline__ bool tile_of(int b, int tiles_m, int tiles_n, int& tm, int& tn) {
  const int T = tiles_m * tiles_n;
  const int per = (T + 7) / 8;
  const int L = (b % 8) * per + b / 8;
  if (L >= T) return false;
  tm = L / tiles_n;
  tn = L % tiles_n;
  return true;
}

// 8 consecutive bf16 of a row starting at element k of a row of length K
// (zero past K); `al` = K % 4 == 0 and 8-byte aligned base (uniform).
__device__ __forceinline__ uint4 load8(const uint16_t* row, int k, int K, bool al) {
  uint4 v = {0u, 0u, 0u, 0u};
  if (al && k + 8 <= K) {
    const uint2 a = *reinterpret_cast<const uint2*>(row + k);
    const uint2 b = *reinterpret_cast<const uint2*>(row + k + 4);
    v.x = a.x; v.y = a.y; v.z = b.x; v.w = b.y;
  } else {
    uint32_t w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int e = 0; e < 8; ++e)
      if (k + e < K) w[e >> 1] |= (uint32_t)row[k + e] << (16 * (e & 1));
    v.x = w[0]; v.y = w[1]; v.z = w[2]; v.w = w[3];
  }
  return v;
}

// Eight consecutive bf16 of a row from element k, raw: with AL (rows 8-byte
// aligned, K % 4 == 0, K >= 8) read at kl = min(k, K - 8), to be moved into
// place by fix8 where they are consumed; else guarded scalar reads.
template <bool AL>
__device__ __forceinline__ uint4 raw8(const uint16_t* row, int k, int K) {
  if (AL) {
    const int kl = min(k, K - 8);
    const uint2 x = *reinterpret_cast<const uint2*>(row + kl);
    const uint2 y = *reinterpret_cast<const uint2*>(row + kl + 4);
    return make_uint4(x.x, x.y, y.x, y.y);
  }
  return load8(row, k, K, false);
}
// The eight values at k from what raw8 read (0 past K): the K tail shifts by
// 4 or lies past K.
template <bool AL>
__device__ __forceinline__ uint4 fix8(uint4 v, int k, int K) {
  if (AL) {
    const int shift = k - min(k, K - 8);  // 0, 4, or >= 8
    if (shift >= 8) return make_uint4(0u, 0u, 0u, 0u);
    if (shift == 4) return make_uint4(v.z, v.w, 0u, 0u);
  }
  return v;
}

// AL: see raw8.  Loads go to clamped in-range rows and keep the raw values;
// rows past M or N are zeroed at the stash (a loaded value that is selected
// on would be turned into a branch around the load, and waited for at once).
template <bool AL>
__global__ __launch_bounds__(512, 4) void k_proj_fwd(const uint16_t* __restrict__ A,
                                                     const uint16_t* __restrict__ Wt,
                                                     float* __restrict__ C, int M, int N, int K) {
  __shared__ __attribute__((aligned(16))) uint16_t As[2][FBM * LDK];  // [m][k]
  __shared__ __attribute__((aligned(16))) uint16_t Bs[2][FBN * LDK];  // [n][k]
  const int tiles_m = (M + FBM - 1) / FBM, tiles_n = (N + FBN - 1) / FBN;
  int tm, tn;
  if (!tile_of(blockIdx.x, tiles_m, tiles_n, tm, tn)) return;
  const int m0 = tm * FBM, n0 = tn * FBN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  // load assignment: A chunks tid and tid + 512 (row = c / 4, k = 8 (c % 4)),
  // Wt chunk tid
  const int ar0 = tid >> 2, ar1 = (tid + 512) >> 2, akc = (tid & 3) * 8;
  const int br = tid >> 2;
  const uint16_t* arow0 = A + (int64_t)min(m0 + ar0, M - 1) * K;
  const uint16_t* arow1 = A + (int64_t)min(m0 + ar1, M - 1) * K;
  const uint16_t* brow = Wt + (int64_t)min(n0 + br, N - 1) * K;
  const bool av0 = m0 + ar0 < M, av1 = m0 + ar1 < M, bv = n0 + br < N;
  const int ns = (K + SK - 1) / SK;
  const uint4 zero = {0u, 0u, 0u, 0u};
  struct Raw {
    uint4 a0, a1, b;
  };
  auto load = [&](int s) -> Raw {
    const int k = min(s, ns - 1) * SK + akc;
    return Raw{raw8<AL>(arow0, k, K), raw8<AL>(arow1, k, K), raw8<AL>(brow, k, K)};
  };
  auto stash = [&](int buf, int s, const Raw& r) {
    const int k = s * SK + akc;
    const bool sv = s < ns;
    *reinterpret_cast<uint4*>(&As[buf][ar0 * LDK + akc]) = (av0 && sv) ? fix8<AL>(r.a0, k, K) : zero;
    *reinterpret_cast<uint4*>(&As[buf][ar1 * LDK + akc]) = (av1 && sv) ? fix8<AL>(r.a1, k, K) : zero;
    *reinterpret_cast<uint4*>(&Bs[buf][br * LDK + akc]) = (bv && sv) ? fix8<AL>(r.b, k, K) : zero;
  };

  f32x16 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;

  auto compute = [&](int buf) {
    const uint16_t* as = As[buf];
    const uint16_t* bs = Bs[buf];
#pragma unroll
    for (int kk = 0; kk < SK; kk += 16) {
      const int kl = kk + 8 * (lane >> 5);
      bf16x8 a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = lds8(as + (wm * 64 + i * 32 + (lane & 31)) * LDK + kl);
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = lds8(bs + (wn * 64 + j * 32 + (lane & 31)) * LDK + kl);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
  };

  // Slab s sits in LDS buffer s % 2; the raw loads of slab t live in register
  // set t % 2 from the top of step t - 2 to the end of step t - 1 (two slabs of
  // products to arrive; the loop is unrolled by two so the sets are fixed
  // registers).
  Raw rs[2];
  rs[0] = load(0);
  rs[1] = load(1);
  stash(0, 0, rs[0]);
  __syncthreads();
  for (int s0 = 0; s0 < ns; s0 += 2) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int s = s0 + u;
      if (s >= ns) break;  // uniform
      rs[u] = load(s + 2);
      compute(u);
      // buffer (s+1)%2 was last read in slab s-1, before the previous barrier
      if (s + 1 < ns) stash(u ^ 1, s + 1, rs[u ^ 1]);
      __syncthreads();
    }
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = n0 + wn * 64 + j * 32 + (lane & 31);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = m0 + wm * 64 + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        if (row < M && col < N) C[(int64_t)row * N + col] = acc[i][j][r];
      }
    }
}

// Forward with binary (spike) input: A given as bits, A_bits [M][wpr] uint32,
// bit k%32 of word k/32 = A[m][k] in {0, 1}: A costs 1/16 of the bf16 path's
// traffic.  bits_to_bf16x8 forms the eight bf16 (0 or 1.0) of one byte of
// bits; the kernels keep it as a 256-entry table in LDS.
__device__ __forceinline__ uint4 bits_to_bf16x8(uint32_t b8) {
  // bit j -> bf16 1.0 (0x3F80) or 0 in element j
  uint32_t w[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const uint32_t lo = (b8 >> (2 * q)) & 1u, hi = (b8 >> (2 * q + 1)) & 1u;
    w[q] = lo * 0x3F80u + hi * 0x3F800000u;
  }
  return make_uint4(w[0], w[1], w[2], w[3]);
}

// AL: as for raw8 (weight rows 8-byte aligned, K % 4 == 0, K >= 8).
// The spike operand stays packed in LDS, two 32-bit words per row and slab:
// A costs 8 bytes of LDS per row and slab instead of 128.  Each lane turns
// the eight bits of its MFMA operand into eight bf16 through a 256-entry
// table in LDS (one 16-byte read) instead of about twenty VALU instructions:
// the matrix cores and the VALU barely overlap on a SIMD, so the expansion's
// VALU time added to the products' (13% faster with the table).  Slabs are
// 64 wide (16 products per wavefront between barriers), so that the loads
// issued two slabs ahead have about a thousand cycles of products to arrive
// from L2.
constexpr int SKB = 64, LDKB = SKB + 8;
template <bool AL>
__global__ __launch_bounds__(512, 4) void k_proj_fwd_bits(const uint32_t* __restrict__ Ab, int wpr,
                                                          const uint16_t* __restrict__ Wt,
                                                          float* __restrict__ C, int M, int N,
                                                          int K) {
  __shared__ uint32_t As[2][FBM][2];                                   // [m][word]: slab bits
  __shared__ __attribute__((aligned(16))) uint16_t Bs[2][FBN * LDKB];  // [n][k]
  __shared__ uint4 lut[256];  // byte -> its eight bits as bf16 0 or 1.0
  const int tiles_m = (M + FBM - 1) / FBM, tiles_n = (N + FBN - 1) / FBN;
  int tm, tn;
  if (!tile_of(blockIdx.x, tiles_m, tiles_n, tm, tn)) return;
  if (threadIdx.x < 256) lut[threadIdx.x] = bits_to_bf16x8(threadIdx.x);  // read after a barrier
  const int m0 = tm * FBM, n0 = tn * FBN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  // A: the thread pair of row ar loads the slab's words ah = 0, 1;
  // Wt: row br, k = 8 (tid % 4) and 32 + 8 (tid % 4) of the slab
  const int ar = tid >> 1, ah = tid & 1;
  const bool av = m0 + ar < M;
  const uint32_t* arow = Ab + (int64_t)min(m0 + ar, M - 1) * wpr;
  const int br = tid >> 2, bkc = (tid & 3) * 8;
  const bool bv = n0 + br < N;
  const uint16_t* brow = Wt + (int64_t)min(n0 + br, N - 1) * K;
  const int ns = (K + SKB - 1) / SKB;
  const int nw = (K + 31) / 32;  // words of a row that hold bits below K

  // Loads go to clamped in-range addresses and keep the raw words; rows past
  // M or N, words past K and bits past K are zeroed at the stash (a load
  // whose value is selected on would be turned into a branch around it, and
  // then waited for at once).  The weights go through raw8 / fix8.
  auto a_bits = [&](int s) -> uint32_t { return arow[min(2 * s + ah, nw - 1)]; };
  auto b_load = [&](int s, int h) -> uint4 {
    return raw8<AL>(brow, min(s, ns - 1) * SKB + 32 * h + bkc, K);
  };
  auto stash = [&](int buf, int s, uint32_t w, uint4 b0, uint4 b1) {
    const int valid = K - 32 * (2 * s + ah);  // bits of this word below K
    if (!av || s >= ns || valid <= 0) w = 0u;
    else if (valid < 32) w &= (1u << valid) - 1u;
    As[buf][ar][ah] = w;
    const bool ok = bv && s < ns;
    b0 = ok ? fix8<AL>(b0, s * SKB + bkc, K) : make_uint4(0u, 0u, 0u, 0u);
    b1 = ok ? fix8<AL>(b1, s * SKB + 32 + bkc, K) : make_uint4(0u, 0u, 0u, 0u);
    *reinterpret_cast<uint4*>(&Bs[buf][br * LDKB + bkc]) = b0;
    *reinterpret_cast<uint4*>(&Bs[buf][br * LDKB + 32 + bkc]) = b1;
  };

  f32x16 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;

  auto compute = [&](int buf) {
    const uint16_t* bs = Bs[buf];
    uint32_t wa[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int row = wm * 64 + i * 32 + (lane & 31);
      wa[i][0] = As[buf][row][0];
      wa[i][1] = As[buf][row][1];
    }
#pragma unroll
    for (int kk = 0; kk < SKB; kk += 16) {
      const int kl = kk + 8 * (lane >> 5);
      bf16x8 a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i)
        a[i] = __builtin_bit_cast(bf16x8, lut[(wa[i][kk >> 5] >> (kl & 31)) & 0xFFu]);
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = lds8(bs + (wn * 64 + j * 32 + (lane & 31)) * LDKB + kl);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
  };

  // Slab s sits in LDS buffer s % 2.  The raw loads of slab t live in
  // register set t % 2: issued at the top of step t - 2 (when that set's
  // previous slab had gone to LDS), stashed at the end of step t - 1, so a
  // load has two slabs of products to arrive.  The loop is unrolled by two
  // so that the sets are fixed registers (no copies, which would wait).
  uint32_t ra[2];
  uint4 rb[2][2];
  ra[0] = a_bits(0);
  rb[0][0] = b_load(0, 0);
  rb[0][1] = b_load(0, 1);
  ra[1] = a_bits(1);
  rb[1][0] = b_load(1, 0);
  rb[1][1] = b_load(1, 1);
  stash(0, 0, ra[0], rb[0][0], rb[0][1]);
  __syncthreads();
  for (int s0 = 0; s0 < ns; s0 += 2) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int s = s0 + u;
      if (s >= ns) break;  // uniform
      ra[u] = a_bits(s + 2);
      rb[u][0] = b_load(s + 2, 0);
      rb[u][1] = b_load(s + 2, 1);
      compute(u);
      // buffer (s+1)%2 was last read in slab s-1, before the previous barrier
      if (s + 1 < ns) stash(u ^ 1, s + 1, ra[u ^ 1], rb[u ^ 1][0], rb[u ^ 1][1]);
      __syncthreads();
    }
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = n0 + wn * 64 + j * 32 + (lane & 31);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = m0 + wm * 64 + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        if (row < M && col < N) C[(int64_t)row * N + col] = acc[i][j][r];
      }
    }
}

// Weight gradient dWt[N][K] = dOut^T A, one split of the reduction over M per
// blockIdx.y.  A block covers 64 output rows n and up to WKB output columns
// k (all of them when K <= WKB), so dOut -- the large fp32 operand -- is read
// exactly once.  The block has eight wavefronts, two per SIMD; wavefront w
// owns the k tiles w, w + 8, w + 16 (WKT of them) for both 32-row halves of
// the n tile: 2 WKT MFMA accumulators of 32 x 32, in the accumulation
// registers.  Slabs of 64 rows of M: each lane loads 4 columns x 2 rows of
// dOut, splits the values into bf16 hi and lo parts and stores them as
// M-contiguous LDS rows [n][m] (double-buffered; the next slab's
// loads are in flight while the current one is multiplied, one barrier per
// slab).  The A operand of a lane -- eight consecutive m of one column k --
// is for spike bits one byte of the column's 32-bit word, expanded through a
// 256-entry LDS table (the bits come in 32-row groups, [M/32][ld], so the
// words of 32 consecutive columns are one 128-byte line); for bf16 A it is
// read from global memory.
// Loads go to clamped in-range addresses and keep the raw values; invalid
// ones are zeroed where they are consumed (zeroing at the load would make
// the load wait at once).
constexpr int WN = 64, WW = 8, WKT = 3, WKB = WW * WKT * 32, WSK = 64, WLD = WSK + 8;

// BITS: A given as bits in 32-row groups, Ab [ceil(M/32)][ldb] (bit m%32 of
// word (m/32, k) = A[m][k]).
template <bool BITS>
__global__ __launch_bounds__(64 * WW, 1) void k_proj_wgrad(const uint16_t* __restrict__ A,
                                                       const uint32_t* __restrict__ Ab, int ldb,
                                                       const float* __restrict__ D,
                                                       float* __restrict__ part, int M, int N,
                                                       int K, int rows_per_split, int tiles_n) {
  __shared__ __attribute__((aligned(16))) uint16_t Dh[2][WN * WLD];  // [n][m]
  __shared__ __attribute__((aligned(16))) uint16_t Dl[2][WN * WLD];  // [n][m]
  __shared__ uint4 lut[256];
  const int tn = blockIdx.x % tiles_n, kb = blockIdx.x / tiles_n;
  const int n0 = tn * WN, kbase = kb * WKB;
  const int mbeg = blockIdx.y * rows_per_split;
  const int mend = min(M, mbeg + rows_per_split);
  const int tid = threadIdx.x, lane = tid & 63, kl = lane & 31;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  if (BITS && tid < 256) {
    // entry b: eight bf16, element e = 1.0 where bit e of b is set
    uint32_t w[4];
#pragma unroll
    for (int j = 0; j < 4; ++j)
      w[j] = ((tid >> (2 * j)) & 1) * 0x3F80u + ((tid >> (2 * j + 1)) & 1) * 0x3F800000u;
    lut[tid] = make_uint4(w[0], w[1], w[2], w[3]);
  }

  f32x16 acc[WKT][2];
#pragma unroll
  for (int j = 0; j < WKT; ++j)
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[j][h][r] = 0.0f;

  // dOut: lane l of wavefront w takes columns n0 + (l & 15) + 16 a (a = 0..3)
  // at rows 2 mp, 2 mp + 1 of the slab, mp = (l >> 4) + 4 w: a wavefront's
  // 4-byte LDS stores then cover 16 consecutive columns x 4 row pairs, which
  // with the 144-byte row pitch are 64 distinct banks (no conflicts).  Each
  // load instruction reads four 64-byte row pieces.
  const int dnl = n0 + (tid & 15), dmp = ((tid & 63) >> 4) + 4 * wave;
  float dq[4][2];
  auto gather = [&](int ms) {
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const float* row = D + (int64_t)min(ms + 2 * dmp + r, M - 1) * N;
#pragma unroll
      for (int a = 0; a < 4; ++a) dq[a][r] = row[min(dnl + 16 * a, N - 1)];
    }
  };
  auto stash = [&](int buf, int ms) {
    const bool r0 = ms + 2 * dmp < mend, r1 = ms + 2 * dmp + 1 < mend;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const bool ok = dnl + 16 * a < N;
      const float x0 = (ok && r0) ? dq[a][0] : 0.0f, x1 = (ok && r1) ? dq[a][1] : 0.0f;
      // hi = x rounded to bf16 (nearest even), lo = the remainder rounded
      const uint32_t hp = pack_bf16(x0, x1);
      const uint32_t lp = pack_bf16(x0 - __uint_as_float(hp << 16), x1 - __uint_as_float(hp & 0xFFFF0000u));
      const int off = ((tid & 15) + 16 * a) * WLD + 2 * dmp;
      *reinterpret_cast<uint32_t*>(&Dh[buf][off]) = hp;
      *reinterpret_cast<uint32_t*>(&Dl[buf][off]) = lp;
    }
  };
  // spike bits of the slab: two words (rows ms .. ms + 31, ms + 32 .. +63)
  // per owned k tile
  uint32_t wcur[WKT][2], wnxt[WKT][2];
  auto bits_load = [&](int ms, uint32_t (&w)[WKT][2]) {
    if (!BITS) return;
#pragma unroll
    for (int j = 0; j < WKT; ++j) {
      const int kc = min(kbase + (wave + WW * j) * 32 + kl, K - 1);
#pragma unroll
      for (int q = 0; q < 2; ++q)
        w[j][q] = Ab[(int64_t)min((ms >> 5) + q, (M - 1) >> 5) * ldb + kc];
    }
  };
  auto b_operand = [&](int j, int ms, int ks, int ml) -> bf16x8 {
    const int kc = kbase + (wave + WW * j) * 32 + kl;
    if (BITS) {
      const uint32_t w = (kc < K && ms + 32 * (ks >> 1) < mend) ? wcur[j][ks >> 1] : 0u;
      return *reinterpret_cast<const bf16x8*>(&lut[(w >> (ml & 31)) & 0xFFu]);
    } else {
      uint32_t w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int m = ms + ml + e;
        const uint32_t v = A[(int64_t)min(m, M - 1) * K + min(kc, K - 1)];
        w[e >> 1] |= ((kc < K && m < mend) ? v : 0u) << (16 * (e & 1));
      }
      const uint4 u = make_uint4(w[0], w[1], w[2], w[3]);
      return *reinterpret_cast<const bf16x8*>(&u);
    }
  };
  // Tiles past K (a wavefront with fewer than WKT) multiply zeros: the slab
  // barrier would make that wavefront wait anyway.
  auto compute = [&](int buf, int ms) {
#pragma unroll
    for (int ks = 0; ks < WSK / 16; ++ks) {
      const int ml = 16 * ks + 8 * (lane >> 5);
      bf16x8 ah[2], al[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        ah[h] = lds8(&Dh[buf][(h * 32 + kl) * WLD + ml]);
        al[h] = lds8(&Dl[buf][(h * 32 + kl) * WLD + ml]);
      }
      if constexpr (BITS) {
        // the operands of the k step first, then every hi product before the
        // lo ones: the two products into one accumulator are six apart
        bf16x8 b[WKT];
#pragma unroll
        for (int j = 0; j < WKT; ++j) b[j] = b_operand(j, ms, ks, ml);
#pragma unroll
        for (int j = 0; j < WKT; ++j)
#pragma unroll
          for (int h = 0; h < 2; ++h)
            acc[j][h] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[h], b[j], acc[j][h], 0, 0, 0);
#pragma unroll
        for (int j = 0; j < WKT; ++j)
#pragma unroll
          for (int h = 0; h < 2; ++h)
            acc[j][h] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[h], b[j], acc[j][h], 0, 0, 0);
      } else {
        // bf16 A: each operand is gathered from global memory just before use
#pragma unroll
        for (int j = 0; j < WKT; ++j) {
          const bf16x8 b = b_operand(j, ms, ks, ml);
#pragma unroll
          for (int h = 0; h < 2; ++h)
            acc[j][h] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[h], b, acc[j][h], 0, 0, 0);
#pragma unroll
          for (int h = 0; h < 2; ++h)
            acc[j][h] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[h], b, acc[j][h], 0, 0, 0);
        }
      }
    }
  };

  // (the first slab's words go through wnxt as well, so the loop is entered
  // the same way from here as from its own end: no load is then still
  // pending at the loop head)
  gather(mbeg);
  bits_load(mbeg, wnxt);
#pragma unroll
  for (int j = 0; j < WKT; ++j) {
    wcur[j][0] = wnxt[j][0];
    wcur[j][1] = wnxt[j][1];
  }
  stash(0, mbeg);
  __syncthreads();  // also publishes the table
  const int ns = (mend - mbeg + WSK - 1) / WSK;
  for (int s = 0; s < ns; ++s) {
    const int buf = s & 1;
    const int ms = mbeg + s * WSK;
    const bool more = s + 1 < ns;
    if (more) {
      gather(ms + WSK);
      bits_load(ms + WSK, wnxt);
    }
    compute(buf, ms);
    if (more) {
      // buffer buf ^ 1 was last read in slab s - 1, before the previous barrier
      stash(buf ^ 1, ms + WSK);
#pragma unroll
      for (int j = 0; j < WKT; ++j) {
        wcur[j][0] = wnxt[j][0];
        wcur[j][1] = wnxt[j][1];
      }
    }
    __syncthreads();
  }
  float* P = part + (int64_t)blockIdx.y * N * K;
#pragma unroll
  for (int j = 0; j < WKT; ++j) {
    const int col = kbase + (wave + WW * j) * 32 + kl;
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = n0 + h * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        if (row < N && col < K) P[(int64_t)row * K + col] = acc[j][h][r];
      }
  }
}

__global__ __launch_bounds__(256) void k_fill_zero(float* __restrict__ p, int64_t count) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0.0f;
}

hipError_t fill_zero(float* p, int64_t count, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, p, count);
  return hipGetLastError();
}

// Sum of the split partials in a fixed order (deterministic); with
// `accumulate` the sum is added to what out holds.
__global__ __launch_bounds__(256) void k_sum_splits(const float* __restrict__ part,
                                                    float* __restrict__ out, int64_t count,
                                                    int splits, int accumulate) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= count) return;
  // eight loads in flight, added in split order (the same sum as one at a time)
  float s = 0.0f;
  int q = 0;
  for (; q + 8 <= splits; q += 8) {
    float v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = part[(int64_t)(q + u) * count + i];
#pragma unroll
    for (int u = 0; u < 8; ++u) s += v[u];
  }
  for (; q < splits; ++q) s += part[(int64_t)q * count + i];
  out[i] = accumulate ? out[i] + s : s;
}

int wgrad_splits(int M) {
  // each split reduces at least 4096 rows: with 16 or more column tiles that
  // fills the chip in one round, and keeps the partial sums small
  int s = (M + 4095) / 4096;
  if (s > 64) s = 64;
  return s < 1 ? 1 : s;
}

}  // namespace

extern "C" {

int32_t hh_proj_forward(const uint16_t* A, const uint16_t* Wt, float* out, int32_t M, int32_t N,
                        int32_t K, void* stream) {
  if (M < 0 || N < 0 || K < 0) return HH_E_SHAPE;
  if (M == 0 || N == 0) return HH_OK;
  if (!out || (K > 0 && (!A || !Wt))) return HH_E_INVALID;
  hipStream_t s = (hipStream_t)stream;
  if (K == 0) return fill_zero(out, (int64_t)M * N, s) == hipSuccess ? HH_OK : HH_E_HIP;
  const int tiles = ((M + FBM - 1) / FBM) * ((N + FBN - 1) / FBN);
  const int blocks = (tiles + 7) / 8 * 8;
  if (K % 4 == 0 && K >= 8 && (uintptr_t)A % 8 == 0 && (uintptr_t)Wt % 8 == 0)
    hipLaunchKernelGGL(k_proj_fwd<true>, dim3(blocks), dim3(512), 0, s, A, Wt, out, M, N, K);
  else
    hipLaunchKernelGGL(k_proj_fwd<false>, dim3(blocks), dim3(512), 0, s, A, Wt, out, M, N, K);
  return hipGetLastError() == hipSuccess ? HH_OK : HH_E_HIP;
}

int32_t hh_proj_forward_bits(const uint32_t* A_bits, int32_t words_per_row, const uint16_t* Wt,
                             float* out, int32_t M, int32_t N, int32_t K, void* stream) {
  if (M < 0 || N < 0 || K < 0) return HH_E_SHAPE;
  if (M == 0 || N == 0) return HH_OK;
  if (!out || (K > 0 && (!A_bits || !Wt))) return HH_E_INVALID;
  if (words_per_row < (K + 31) / 32) return HH_E_SHAPE;
  hipStream_t s = (hipStream_t)stream;
  if (K == 0) return fill_zero(out, (int64_t)M * N, s) == hipSuccess ? HH_OK : HH_E_HIP;
  const int tiles = ((M + FBM - 1) / FBM) * ((N + FBN - 1) / FBN);
  const int blocks = (tiles + 7) / 8 * 8;
  if (K % 4 == 0 && K >= 8 && (uintptr_t)Wt % 8 == 0)
    hipLaunchKernelGGL(k_proj_fwd_bits<true>, dim3(blocks), dim3(512), 0, s, A_bits, words_per_row,
                       Wt, out, M, N, K);
  else
    hipLaunchKernelGGL(k_proj_fwd_bits<false>, dim3(blocks), dim3(512), 0, s, A_bits, words_per_row,
                       Wt, out, M, N, K);
  return hipGetLastError() == hipSuccess ? HH_OK : HH_E_HIP;
}

size_t hh_proj_wgrad_workspace(int32_t M, int32_t N, int32_t K) {
  if (M <= 0 || N <= 0 || K <= 0) return 0;
  return (size_t)wgrad_splits(M) * (size_t)K * (size_t)N * sizeof(float);
}

int32_t hh_proj_wgrad(const uint16_t* A, const float* dOut, float* dWt, int32_t accumulate,
                      int32_t M, int32_t N, int32_t K, void* workspace, size_t workspace_bytes,
                      void* stream) {
  if (M < 0 || N < 0 || K < 0) return HH_E_SHAPE;
  if (N == 0 || K == 0) return HH_OK;
  if (!dWt || (M > 0 && (!A || !dOut))) return HH_E_INVALID;
  hipStream_t s = (hipStream_t)stream;
  if (M == 0) {
    if (accumulate) return HH_OK;
    return fill_zero(dWt, (int64_t)N * K, s) == hipSuccess ? HH_OK : HH_E_HIP;
  }
  const size_t need = hh_proj_wgrad_workspace(M, N, K);
  if (!workspace || workspace_bytes < need) return HH_E_SHAPE;
  const int splits = wgrad_splits(M);
  int rows = (M + splits - 1) / splits;
  rows = (rows + SK - 1) / SK * SK;
  const int tiles_n = (N + WN - 1) / WN;
  const int blocks = tiles_n * ((K + WKB - 1) / WKB);
  float* part = (float*)workspace;
  hipLaunchKernelGGL(k_proj_wgrad<false>, dim3(blocks, splits), dim3(64 * WW), 0, s, A, nullptr, 0,
                     dOut, part, M, N, K, rows, tiles_n);
  const int64_t count = (int64_t)K * N;
  hipLaunchKernelGGL(k_sum_splits, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, part,
                     dWt, count, splits, accumulate ? 1 : 0);
  return hipGetLastError() == hipSuccess ? HH_OK : HH_E_HIP;
}

int32_t hh_proj_wgrad_bits(const uint32_t* A_bits, int32_t ld, const float* dOut, float* dWt,
                           int32_t accumulate, int32_t M, int32_t N, int32_t K, void* workspace,
                           size_t workspace_bytes, void* stream) {
  if (M < 0 || N < 0 || K < 0) return HH_E_SHAPE;
  if (N == 0 || K == 0) return HH_OK;
  if (!dWt || (M > 0 && (!A_bits || !dOut))) return HH_E_INVALID;
  if (ld < K) return HH_E_SHAPE;
  hipStream_t s = (hipStream_t)stream;
  if (M == 0) {
    if (accumulate) return HH_OK;
    return fill_zero(dWt, (int64_t)N * K, s) == hipSuccess ? HH_OK : HH_E_HIP;
  }
  const size_t need = hh_proj_wgrad_workspace(M, N, K);
  if (!workspace || workspace_bytes < need) return HH_E_SHAPE;
  const int splits = wgrad_splits(M);
  int rows = (M + splits - 1) / splits;
  rows = (rows + SK - 1) / SK * SK;
  const int tiles_n = (N + WN - 1) / WN;
  const int blocks = tiles_n * ((K + WKB - 1) / WKB);
  float* part = (float*)workspace;
  hipLaunchKernelGGL(k_proj_wgrad<true>, dim3(blocks, splits), dim3(64 * WW), 0, s, nullptr, A_bits,
                     ld, dOut, part, M, N, K, rows, tiles_n);
  const int64_t count = (int64_t)K * N;
  hipLaunchKernelGGL(k_sum_splits, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, part,
                     dWt, count, splits, accumulate ? 1 : 0);
  return hipGetLastError() == hipSuccess ? HH_OK : HH_E_HIP;
}

}  // extern "C"
