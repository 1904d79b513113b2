// hh_net.hip -- recurrent network of HH neurons with conductance synapses
// delivered through a CSR connectivity (Results, cortical network; sparse
// synapses with indirect addressing).
//
// Time loop: one persistent cooperative kernel keeps every neuron's state in
// registers for the whole run.  Per step:
//   A  each lane advances its neuron with the conductances held over the
//      step, decays them, adds its external Poisson event, and detects an
//      upward threshold crossing;
//      the block compacts its spiking neurons (wave ballot, mbcnt rank, one
//      LDS atomic per wave) and scatters their CSR rows into the arrival
//      accumulator of this step (64-bit fixed point, 2^-40 mS/cm^2 per unit,
//      so the sum does not depend on the order of arrival);
//   -- grid barrier --
//   B  each lane takes (and clears) its own arrivals into g_e, g_i.
// Two accumulator buffers alternate between steps, so one barrier per step
// suffices.  With per-synapse delays of up to D steps the accumulators form
// a ring of D + 1 slots indexed by absolute time: a step reads and clears
// the slot of its own time and scatters into the slots 1..D steps ahead, so
// reads and writes of one step never meet; arrivals still in flight at the
// end of a call stay in the ring for the next call.
//
// A population of B copies of one network (n = N B elements, copy b holding
// elements b N .. b N + N - 1) shares the CSR of N rows: a spike of element
// b N + j goes through row j to targets b N + col.  The copies are the
// paper's parallel simulations of one network on one device; each draws
// its own external and background streams, keyed by the element index.
//
// hh_syn_propagate runs the same delivery once, outside the time loop, as
// three kernels: global compaction, the scatter (binned by target range when
// the rows are sorted, else one wavefront per spiking row), apply.
#include <stdlib.h>
#include <string.h>

#include <cmath>

#include "hh_barrier.h"
#include "hh_internal.h"

using namespace hhk;

namespace {

constexpr float kFix = 1099511627776.0f;        // 2^40
constexpr float kUnfix = 9.094947017729282e-13f;  // 2^-40
constexpr int kNetBlock = 512;      // threads per block of the network kernel
constexpr int kNetBlockWide = 1024; // for large grids with the pull delivery
constexpr int64_t kWideMinBlocks = 128;  // in blocks of kNetBlock
constexpr int kSegRange = 512;      // targets per range of the segment table
// Grids of at least this many blocks synchronize with the flag-array barrier
// (measured per step: 3.3 against 3.7 us at 75 blocks, 10.5 against 19.0 us
// at 446); smaller ones with the single arrival counter (1.2 against 2.0 us
// at 8 blocks).
constexpr unsigned kFlagBarrierMin = 32;

struct NetArgs {
  float* state;
  int64_t n;
  int64_t N;                // elements per copy (rows of the shared CSR)
  int32_t B;                // copies
  const int64_t* row_ptr;
  const int32_t* col;
  const float* w;
  float w_scale;
  const uint8_t* ext_mask;
  uint32_t ext_thresh;
  float w_ext;
  uint64_t ext_seed;
  const float* i_const;
  int64_t t0;
  int32_t nsteps;
  uint32_t* spikes;
  int64_t words;
  unsigned long long* acc;  // [2 buffers][2 (e, i)][n], or with delays [R slots][2][n]
  const uint8_t* delay;     // per-synapse delays in steps (null: 1)
  int32_t R;                // ring slots (max delay + 1) when delay is set
  // background input (Methods, cortical network): drawn per step when bg != 0
  int32_t bg;
  float mu, sigma, bg_lam, bg_p0;
  int32_t bg_kmax;
  uint64_t seed;
  // pull delivery (one-step delays, rows sorted by target): the spiking rows
  // of copy c at step k in plist[k & 1][c][0 .. pcount[k % 3][c]), and the
  // segment table of the rows by 512-target ranges
  int32_t* plist;
  unsigned* pcount;
  const int32_t* seg;
  int32_t seg_R;
  unsigned* bar;            // [0] arrivals (monotonic within a launch)
  int32_t* flags;           // [0] first non-finite neuron, [1] timeout
  uint32_t spin_limit;
};

__device__ __forceinline__ void deliver_row(const int64_t* __restrict__ row_ptr,
                                            const int32_t* __restrict__ col,
                                            const float* __restrict__ w, float scale40, int j,
                                            int base, unsigned long long* acc_e,
                                            unsigned long long* acc_i, int lane0, int stride) {
  const int64_t r0 = row_ptr[j], r1 = row_ptr[j + 1];
  for (int64_t q = r0 + lane0; q < r1; q += stride) {
    const int32_t tgt = base + col[q];
    const float wv = w[q];
    const unsigned long long inc = (unsigned long long)__float2ull_rn(fabsf(wv) * scale40);
    atomicAdd(wv > 0.0f ? &acc_e[tgt] : &acc_i[tgt], inc);
  }
}

// Inclusive prefix sum of v[0..cnt) in LDS, cnt <= blockDim (Hillis-Steele;
// short lists are summed by one lane).  Ends with a barrier.
__device__ void block_inclusive_scan(int* v, int cnt) {
  if (cnt <= 32) {
    if (threadIdx.x == 0)
      for (int e = 1; e < cnt; ++e) v[e] += v[e - 1];
    __syncthreads();
    return;
  }
  for (int off = 1; off < cnt; off <<= 1) {
    int x = 0;
    const int t = threadIdx.x;
    if (t < cnt && t >= off) x = v[t - off];
    __syncthreads();
    if (t < cnt && t >= off) v[t] += x;
    __syncthreads();
  }
}

// Scatter of `total` synaptic events of the block's spiking rows: lane t
// takes events t, t + B, t + 2B, ... (B = block size), issuing up to 16
// independent (col, w) loads before its atomics so the loads overlap.
// s_base holds each spiking row's copy offset (b N), added to its targets.
// DELAY: the events go to the ring slot (now + d) of their synapse's delay
// d (clamped to [1, R - 1], so the slot always lies in the ring); acc_e is
// then the ring's base and `now` the current time's slot.
template <bool DELAY = false, bool BATCH = false>
__device__ __forceinline__ void scatter_flat(const int32_t* __restrict__ col,
                                             const float* __restrict__ w, float scale40,
                                             const int64_t* s_r0, const int* s_pre,
                                             const int* s_base, int cnt,
                                             int total, unsigned long long* acc_e,
                                             unsigned long long* acc_i,
                                             const uint8_t* __restrict__ delay = nullptr,
                                             int now = 0, int R = 2, int64_t n = 0) {
  constexpr int U = 16;
  const int B = blockDim.x;
  for (int x0 = threadIdx.x; x0 < total; x0 += U * B) {
    int32_t tg[U];
    float wv[U];
    int sl[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int x = x0 + u * B;
      tg[u] = -1;
      wv[u] = 0.0f;
      sl[u] = 0;
      if (x < total) {
        // row e: first e with s_pre[e] > x
        int lo = 0, hi = cnt - 1;
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (s_pre[mid] > x) hi = mid;
          else lo = mid + 1;
        }
        const int before = lo ? s_pre[lo - 1] : 0;
        const int64_t q = s_r0[lo] + (x - before);
        tg[u] = BATCH ? s_base[lo] + col[q] : col[q];
        wv[u] = w[q];
        if constexpr (DELAY) {
          const int d = min(max((int)delay[q], 1), R - 1);
          sl[u] = now + d >= R ? now + d - R : now + d;
        }
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (tg[u] >= 0) {
        const unsigned long long inc = (unsigned long long)__float2ull_rn(fabsf(wv[u]) * scale40);
        if constexpr (DELAY) {
          unsigned long long* slot = acc_e + (int64_t)sl[u] * 2 * n;
          atomicAdd(wv[u] > 0.0f ? &slot[tg[u]] : &slot[n + tg[u]], inc);
        } else {
          atomicAdd(wv[u] > 0.0f ? &acc_e[tg[u]] : &acc_i[tg[u]], inc);
        }
      }
    }
  }
}

// Pull delivery of one step's spikes of one copy into the block's own
// targets: the block owning elements [lo, lo + BS) reads the copy's
// list of spiking rows, then each row's span of targets that covers the
// block's window [x0, x1) of the copy (table ranges r0..r1 of the segment
// table of the rows sorted by target), and adds the events inside the window
// into LDS accumulators, one per element and sign (element = col + ldsoff).
// No device atomics and no accumulator buffers; the integer sums equal those
// of the push delivery bit for bit.  The list and its count were written by
// other blocks before the last grid barrier: they are read with device-scope
// loads.  s_a and s_len are staging arrays of BS entries; the
// accumulators are complete when it returns.
template <int BS>
__device__ void pull_deliver(const int32_t* list, const unsigned* countp, int64_t N,
                             const int32_t* __restrict__ seg, int R, int r0, int r1, int x0,
                             int x1, int ldsoff, const int64_t* __restrict__ row_ptr,
                             const int32_t* __restrict__ col, const float* __restrict__ w,
                             float scale40, unsigned long long* s_e, unsigned long long* s_i,
                             int64_t* s_a, int* s_len) {
  const int tid = threadIdx.x;
  // the count and the first BS entries in one round trip
  unsigned cnt = __hip_atomic_load(countp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const int32_t spec = tid < N ? __hip_atomic_load(&list[tid], __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT)
                               : 0;
  // every lane reads the same final count (no block adds to it until the
  // barrier after this one); thread 0's copy is still broadcast so that the
  // loop below, which holds barriers, is uniform over the block by
  // construction
  __shared__ unsigned s_pc;
  if (tid == 0) s_pc = (unsigned)min((int64_t)cnt, N);
  __syncthreads();
  cnt = s_pc;
  constexpr int G = 16;  // lanes per row span
  for (unsigned c0 = 0; c0 < cnt; c0 += BS) {
    const unsigned e = c0 + tid;
    if (e < cnt) {
      const int32_t src = c0 == 0 ? spec
                                  : __hip_atomic_load(&list[e], __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT);
      const int32_t* sj = seg + (int64_t)src * (R + 1);
      const int32_t s0 = sj[r0], s1 = sj[r1 + 1];
      s_a[tid] = row_ptr[src] + s0;
      s_len[tid] = s1 - s0;
    }
    __syncthreads();
    const int rows = (int)min(cnt - c0, (unsigned)BS);
    for (int x = tid / G; x < rows; x += BS / G) {
      const int64_t a = s_a[x];
      const int len = s_len[x];
      for (int b0 = 0; b0 < len; b0 += 4 * G) {
        int32_t c[4];
        float wv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int q = b0 + u * G + (tid & (G - 1));
          c[u] = q < len ? col[a + q] : -1;
          wv[u] = q < len ? w[a + q] : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          if (c[u] >= x0 && c[u] < x1) {
            const unsigned long long inc =
                (unsigned long long)__float2ull_rn(fabsf(wv[u]) * scale40);
            const int t = c[u] + ldsoff;
            atomicAdd(wv[u] > 0.0f ? &s_e[t] : &s_i[t], inc);
          }
        }
      }
    }
    __syncthreads();
  }
}

// The block's targets in copy c: window [x0, x1) of the copy's N elements,
// its table ranges r0..r1, and the offset from copy-local target to LDS slot.
struct PullWin {
  int x0, x1, r0, r1, ldsoff;
};
__device__ __forceinline__ PullWin pull_window(int64_t lo, int64_t hi, int64_t c, int64_t N) {
  PullWin p;
  const int64_t base = c * N;
  p.x0 = (int)max(lo - base, (int64_t)0);
  p.x1 = (int)min(hi - base, N);
  p.r0 = p.x0 / kSegRange;
  p.r1 = (p.x1 - 1) / kSegRange;
  p.ldsoff = (int)(base - lo);
  return p;
}

// One step of neuron_step's arithmetic, reordered so that the previous
// step's synaptic arrivals (read-and-clear atomics issued by the caller) are
// needed only after the gates: the gate update, which reads V and the old
// gates only, hides the atomics' latency.  Same operations as neuron_step,
// so the same results.
template <class S>
__device__ __forceinline__ void net_update(const KModel& M, const LaneRates<S::kNG>& L, float dtC,
                                           float& vh, float& vl, float (&p)[ng1<S::kNG>],
                                           float I, float& ge, float& gi,
                                           unsigned long long ae, unsigned long long ai) {
  constexpr int NG = S::kNG;
  const float V = vh;
  float po[ng1<NG>];
#pragma unroll
  for (int g = 0; g < NG; ++g) po[g] = p[g];
  // gates by exponential Euler at V_t
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    const float r0 = rate_eval<false>(S::form(M, g, 0), L.r[g][0], V, nullptr);
    const float r1 = rate_eval<false>(S::form(M, g, 1), L.r[g][1], V, nullptr);
    if (S::kind(M, g) == KIND_AB) {
      const float sr = r0 + r1;
      p[g] = gate_update(p[g], r0 * rcp(sr), ex2(sr * M.kdt));
    } else {
      // slow (p_inf, 1/tau) gates: 1 - e from the series, as in neuron_step
      p[g] = fmaf(r0 - p[g], one_minus_exp_neg(r1 * M.dt), p[g]);
    }
  }
  // arrivals of the previous step's spikes
  ge += (float)ae * kUnfix;
  gi += (float)ai * kUnfix;
  // channel terms at the start-of-step gates
  float gsum = ge + gi;
  float esum = fmaf(ge, M.E_e, gi * M.E_i);
#pragma unroll
  for (int c = 0; c < kMaxCh; ++c) {
    if (c >= S::nch(M)) break;
    float eta = M.gbar[c];
#pragma unroll
    for (int g = 0; g < NG; ++g) {
      const int e = S::cexp(M, c, g);
      if (e) eta *= ipow(po[g], e);
    }
    gsum += eta;
    esum = fmaf(eta, M.E[c], esum);
  }
  // membrane
  float dv;
  if (M.v_method == VFE) {
    const float iion = fmaf(gsum, vl, fmaf(gsum, V, -esum));
    dv = dtC * (I - iion);
  } else {
    const float vinf = (I + esum) * rcp(gsum);
    dv = ((V - vinf) + vl) * expm1_neg(gsum * dtC);
  }
  add_to_v(vh, vl, dv);
}

// BATCH: more than one copy of the network (B > 1); a single network skips
// the copy offsets entirely.  PULL: one-step delays and a segment table:
// delivery by pull_deliver instead of the scatter (with BATCH, N >= 512, so
// that a block's elements span at most two copies).
template <class S, bool DELAY, bool BATCH, bool PULL = false, int BS = kNetBlock>
__global__ __launch_bounds__(BS) void k_net(KModel M, NetArgs A) {
  static_assert(!(PULL && DELAY), "pull delivery: one-step delays");
  constexpr int NG = S::kNG;
  __shared__ int s_pre[BS];
  __shared__ int s_base[BS];
  __shared__ int64_t s_r0[BS];
  __shared__ unsigned long long s_ae[PULL ? BS : 1], s_ai[PULL ? BS : 1];
  __shared__ int s_cnt;
  __shared__ unsigned s_gbase[2];
  __shared__ int s_ccnt[2];
  __shared__ int s_ok;
  const int64_t n = A.n;
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const bool act = i < n;
  const int64_t ii = act ? i : n - 1;
  const int lane = threadIdx.x & 63;
  const int64_t w0 = (i - lane) >> 5;

  LaneRates<NG> L;
  load_rates<S>(M, nullptr, 0, 1, L);
  const float dtC = M.dt / M.C;
  const int64_t row_ge = (int64_t)(1 + NG) * n, row_gi = (int64_t)(2 + NG) * n;
  const int64_t row_lo = (int64_t)(3 + NG) * n;
  float vh = A.state[ii], vl = A.state[row_lo + ii];
  float p[ng1<NG>];
#pragma unroll
  for (int g = 0; g < NG; ++g) p[g] = A.state[(int64_t)(1 + g) * n + ii];
  float ge = A.state[row_ge + ii], gi = A.state[row_gi + ii];
  const float I = A.i_const ? A.i_const[ii] : 0.0f;
  // element ii is neuron j of copy b: row j of the shared CSR, targets
  // offset by b N
  const int64_t jj = BATCH ? ii % A.N : ii;
  const int my_base = (int)(ii - jj);
  const bool driven = A.ext_mask && act && A.ext_mask[jj];
  const float scale40 = A.w_scale * kFix;
  unsigned gen = 0;
  // this neuron's CSR row, read once: a spiking lane hands it to the
  // block's scatter without another dependent load
  const int64_t my_r0 = A.row_ptr[jj];
  const int my_len = (int)(A.row_ptr[jj + 1] - my_r0);
  int done = 0;  // steps whose barrier completed
  // ring slot of the current time (DELAY), advanced once per step
  int now = DELAY ? (int)(A.t0 % A.R) : 0;
  // the block's elements [lo, hi) and the copies cf..cl they belong to (PULL)
  const int64_t lo = (int64_t)blockIdx.x * BS, hi = min(lo + (int64_t)BS, n);
  const int64_t cf = lo / A.N, cl = (hi - 1) / A.N;  // cl <= cf + 1 (N >= BS)
  const int my_c = (int)(ii / A.N - cf);              // 0 or 1
  if constexpr (PULL) {
    s_ae[threadIdx.x] = 0ull;
    s_ai[threadIdx.x] = 0ull;
  }
  auto pull_all = [&](int step) {
    for (int64_t c = cf; c <= cl; ++c) {
      const PullWin pw = pull_window(lo, hi, c, A.N);
      pull_deliver<BS>(A.plist + ((int64_t)(step & 1) * n + c * A.N),
                   A.pcount + (int64_t)(step % 3) * A.B + c, A.N, A.seg, A.seg_R, pw.r0, pw.r1,
                   pw.x0, pw.x1, pw.ldsoff, A.row_ptr, A.col, A.w, scale40, s_ae, s_ai, s_r0,
                   s_pre);
    }
  };

  for (int k = 0; k < A.nsteps; ++k) {
    const int64_t t = A.t0 + k;
    const float V = vh;
    // arrivals due at this step (those due at the first step of a launch
    // were folded into the state at the end of the previous launch, or the
    // ring was cleared for a run that starts at t0 = 0)
    unsigned long long ae = 0ull, ai = 0ull;
    if constexpr (PULL) {
      if (k > 0) {
        pull_all(k - 1);
        ae = s_ae[threadIdx.x];
        ai = s_ai[threadIdx.x];
        s_ae[threadIdx.x] = 0ull;
        s_ai[threadIdx.x] = 0ull;
      }
    } else if (k > 0 && act) {
      unsigned long long* pe = DELAY ? A.acc + (int64_t)now * 2 * n
                                     : A.acc + (int64_t)((k - 1) & 1) * 2 * n;
      ae = atomicExch(&pe[i], 0ull);
      ai = atomicExch(&pe[n + i], 0ull);
    }
    const float Ik = A.bg ? background_current(A.seed, (uint32_t)ii, (uint64_t)t, A.bg_lam, A.bg_p0,
                                               A.bg_kmax, A.mu, A.sigma)
                          : I;
    net_update<S>(M, L, dtC, vh, vl, p, Ik, ge, gi, ae, ai);
    const bool spk = act && (V < M.v_th) && (vh >= M.v_th);
    ge *= M.decay_e;
    gi *= M.decay_i;
    if (driven && event_word(A.ext_seed, (uint32_t)i, (uint64_t)(t + 1)) < A.ext_thresh) ge += A.w_ext;

    // compaction of this block's spiking neurons
    if (threadIdx.x == 0) s_cnt = 0;
    __syncthreads();
    const uint64_t b = __ballot(spk);
    if (A.spikes && lane == 0 && w0 < A.words) {
      uint32_t* row = A.spikes + (int64_t)k * A.words;
      row[w0] = (uint32_t)b;
      if (w0 + 1 < A.words) row[w0 + 1] = (uint32_t)(b >> 32);
    }
    int myslot = -1;  // this lane's rank among the block's spiking neurons (of its copy)
    if constexpr (!PULL) {
      if (b) {
        int base = 0;
        if (lane == 0) base = atomicAdd(&s_cnt, __popcll(b));
        base = __shfl(base, 0);
        if (spk) {
          myslot = base + __builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32),
                                                    __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0u));
          // flatten the (row, synapse) pairs of all spiking rows of the block
          s_r0[myslot] = my_r0;
          s_pre[myslot] = my_len;
          if constexpr (BATCH) s_base[myslot] = my_base;
        }
      }
    } else {
      // ranks per copy: the block's elements belong to copy cf + 0 or cf + 1
      if (threadIdx.x < 2) s_ccnt[threadIdx.x] = 0;
      // the counts of step k - 2 have been read by every block (before the
      // last barrier) and are next added to at step k + 1: clear them now
      if (blockIdx.x == 0)
        for (int c = threadIdx.x; c < A.B; c += BS)
          __hip_atomic_store(A.pcount + (int64_t)((k + 1) % 3) * A.B + c, 0u, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
      __syncthreads();
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const uint64_t bh = __ballot(spk && my_c == h);
        if (bh) {
          int base = 0;
          if (lane == 0) base = atomicAdd(&s_ccnt[h], __popcll(bh));
          base = __shfl(base, 0);
          if (spk && my_c == h)
            myslot = base + __builtin_amdgcn_mbcnt_hi((uint32_t)(bh >> 32),
                                                      __builtin_amdgcn_mbcnt_lo((uint32_t)bh, 0u));
        }
      }
      __syncthreads();
      // each copy's spiking rows of the block go to its list at one offset
      if (threadIdx.x < 2 && s_ccnt[threadIdx.x] > 0)
        s_gbase[threadIdx.x] = __hip_atomic_fetch_add(
            A.pcount + (int64_t)(k % 3) * A.B + cf + threadIdx.x, (unsigned)s_ccnt[threadIdx.x],
            __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __syncthreads();
      if (myslot >= 0)
        A.plist[(int64_t)(k & 1) * n + (cf + my_c) * A.N + s_gbase[my_c] + myslot] = (int32_t)jj;
    }
    __syncthreads();
    const int cnt = s_cnt;
    if (!PULL && cnt > 0) {
      block_inclusive_scan(s_pre, cnt);
      const int total = s_pre[cnt - 1];
      if constexpr (DELAY) {
        scatter_flat<true, BATCH>(A.col, A.w, scale40, s_r0, s_pre, s_base, cnt, total, A.acc,
                                  nullptr, A.delay, now, A.R, n);
      } else {
        unsigned long long* acc_e = A.acc + (int64_t)(k & 1) * 2 * n;
        scatter_flat<false, BATCH>(A.col, A.w, scale40, s_r0, s_pre, s_base, cnt, total, acc_e,
                                   acc_e + n);
      }
    }

    const bool passed = gridDim.x >= kFlagBarrierMin
                            ? grid_barrier3(A.bar, gridDim.x, gen, A.spin_limit, A.flags, &s_ok)
                            : grid_barrier(A.bar, gridDim.x, gen, A.spin_limit, A.flags, &s_ok);
    if (!passed) break;
    done = k + 1;
    if constexpr (DELAY) now = now + 1 == A.R ? 0 : now + 1;
  }
  // the arrivals due at the step after the last one
  if constexpr (PULL) {
    if (done > 0) {  // uniform over the block: its threads passed the same barriers
      pull_all(done - 1);
      ge += (float)s_ae[threadIdx.x] * kUnfix;
      gi += (float)s_ai[threadIdx.x] * kUnfix;
    }
  } else if (done > 0 && act) {
    unsigned long long* pe = DELAY ? A.acc + (int64_t)now * 2 * n
                                   : A.acc + (int64_t)((done - 1) & 1) * 2 * n;
    ge += (float)atomicExch(&pe[i], 0ull) * kUnfix;
    gi += (float)atomicExch(&pe[n + i], 0ull) * kUnfix;
  }

  if (!act) return;
  A.state[i] = vh;
  A.state[row_lo + i] = vl;
#pragma unroll
  for (int g = 0; g < NG; ++g) A.state[(int64_t)(1 + g) * n + i] = p[g];
  A.state[row_ge + i] = ge;
  A.state[row_gi + i] = gi;
  if (!__builtin_isfinite(vh + vl + ge + gi)) atomicMin(&A.flags[0], (int32_t)i);
}

// zero fill of the delay ring (a fill kernel rather than a memset, so that
// a captured stream replays it correctly)
__global__ void k_zero64(unsigned long long* p, int64_t count) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0ull;
}

// the barrier words and the pull delivery's list counts (3 steps x B copies)
__global__ void k_net_reset(unsigned* bar, int bar_words, unsigned* pcount, int count) {
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < bar_words; c += gridDim.x * blockDim.x)
    bar[c] = 0u;
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < count; c += gridDim.x * blockDim.x)
    pcount[c] = 0u;
}

// ---- one-shot delivery -----------------------------------------------------
__global__ void k_zero_u32(unsigned* p, int count) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < count) p[j] = 0u;
}

__global__ __launch_bounds__(256) void k_compact(const uint32_t* __restrict__ bits, int64_t n,
                                                 int32_t* __restrict__ list, unsigned* count) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const bool spk = i < n && ((bits[i >> 5] >> (i & 31)) & 1u);
  const uint64_t b = __ballot(spk);
  if (!b) return;
  const int lane = threadIdx.x & 63;
  unsigned base = 0;
  if (lane == 0) base = atomicAdd(count, (unsigned)__popcll(b));
  base = __shfl(base, 0);
  if (spk) {
    const unsigned rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32),
                                                    __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0u));
    list[base + rank] = (int32_t)i;
  }
}

// One wavefront per spiking source row.
__global__ __launch_bounds__(256) void k_scatter(const int32_t* __restrict__ list,
                                                 const unsigned* count, int N,
                                                 const int64_t* __restrict__ row_ptr,
                                                 const int32_t* __restrict__ col,
                                                 const float* __restrict__ w, float scale40,
                                                 unsigned long long* acc_e,
                                                 unsigned long long* acc_i) {
  const unsigned cnt = *count;
  const int lane = threadIdx.x & 63;
  const unsigned waves = gridDim.x * (blockDim.x >> 6);
  for (unsigned e = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); e < cnt; e += waves) {
    const int src = list[e], j = src % N;
    deliver_row(row_ptr, col, w, scale40, j, src - j, acc_e, acc_i, lane, 64);
  }
}

// ---- binned one-shot delivery ----------------------------------------------
// With the rows sorted by target, the delivery is split by target range: a
// block owns kBinSpan table ranges of targets and a chunk of the spiking rows, adds the
// rows' events that fall in its range into LDS accumulators (one LDS atomic
// per event), and then adds each touched accumulator to the global one with
// a single device-scope atomic.  Every event is read once; the global atomics
// fall from one per event (contention on a few thousand cache lines) to one
// per target and chunk.  The sums are integers, so the result equals the
// per-event delivery's bit for bit.
constexpr int kBinSpan = 2;       // table ranges per one-shot block (1,024 targets)
constexpr int kSegChunk = 2048;   // spiking rows per block
constexpr int kBinBlock = 512;    // threads per block: 32 groups of 16 lanes
constexpr int kBinGroup = 16;     // lanes that share one row's segment
constexpr int kBinUnroll = 8;     // loads in flight per lane (128 events per pass)

// Per row: validity (row_ptr non-decreasing within [0, nnz], starting at 0
// and ending at nnz; every column in [0, N)), sortedness, and -- when seg is
// given -- the offsets of the range boundaries.  flags bit 0: some row is
// not sorted; bit 1: the CSR is invalid (nothing past a bad row_ptr entry
// is read).
__global__ __launch_bounds__(256) void k_csr_segments(const int64_t* __restrict__ row_ptr,
                                                      const int32_t* __restrict__ col, int64_t N,
                                                      int64_t nnz, int R, int32_t* __restrict__ seg,
                                                      int* __restrict__ flags) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= N) return;
  const int64_t r0 = row_ptr[j], r1 = row_ptr[j + 1];
  if (r0 < 0 || r1 < r0 || r1 > nnz || (j == 0 && r0 != 0) || (j == N - 1 && r1 != nnz)) {
    atomicOr(flags, 2);
    return;
  }
  int32_t* sj = seg ? seg + j * (int64_t)(R + 1) : nullptr;
  int r = 0;
  int32_t prev = -1;
  bool unsorted = false, bad = false;
  for (int64_t q = r0; q < r1; ++q) {
    const int32_t c = col[q];
    unsorted |= c < prev;
    bad |= c < 0 || c >= N;
    prev = c;
    if (sj)
      while (r <= R && (int64_t)r * kSegRange <= c) sj[r++] = (int32_t)(q - r0);
  }
  if (sj)
    while (r <= R) sj[r++] = (int32_t)(r1 - r0);
  if (unsorted || bad) atomicOr(flags, (unsorted ? 1 : 0) | (bad ? 2 : 0));
}

// Grid: R ranges x chunks blocks in one dimension.  Consecutive hardware
// block ids go to the eight XCDs in turn; the remap gives each XCD a run of
// consecutive logical blocks, i.e. neighbouring ranges of the same chunk, so
// the cache lines two neighbouring segments share are fetched into one L2.
__global__ __launch_bounds__(kBinBlock) void k_scatter_binned(
    const int32_t* __restrict__ list, const unsigned* count, const int64_t* __restrict__ row_ptr,
    const int32_t* __restrict__ col, const float* __restrict__ w, const int32_t* __restrict__ seg,
    int R, float scale40, unsigned long long* __restrict__ acc_e,
    unsigned long long* __restrict__ acc_i, int64_t n) {
  constexpr int kSpan = kBinSpan * kSegRange;  // targets per block
  __shared__ unsigned long long se[kSpan], si[kSpan];
  __shared__ int64_t m_a[kSegChunk];
  __shared__ int32_t m_len[kSegChunk];
  const unsigned nb = gridDim.x, bid = blockIdx.x;
  const unsigned xcd = bid & 7u, idx = bid >> 3, per = nb >> 3, rem = nb & 7u;
  const unsigned logical = xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
  const int spans = (R + kBinSpan - 1) / kBinSpan;
  const int rs = (int)(logical % (unsigned)spans);
  const int r = rs * kBinSpan, r_end = min(r + kBinSpan, R);  // table ranges [r, r_end)
  const unsigned e0 = (logical / (unsigned)spans) * (unsigned)kSegChunk;
  const unsigned cnt = *count;
  if (e0 >= cnt) return;  // uniform: the whole block leaves
  const int rows = (int)min(cnt - e0, (unsigned)kSegChunk);
  const int tid = threadIdx.x;
  for (int t = tid; t < kSpan; t += kBinBlock) se[t] = si[t] = 0ull;
  // the chunk's segments for this range, four rows per thread loaded together
  {
    int src[kSegChunk / kBinBlock];
#pragma unroll
    for (int u = 0; u < kSegChunk / kBinBlock; ++u) {
      const int i = tid + u * kBinBlock;
      src[u] = i < rows ? list[e0 + i] : 0;
    }
#pragma unroll
    for (int u = 0; u < kSegChunk / kBinBlock; ++u) {
      const int i = tid + u * kBinBlock;
      if (i < rows) {
        const int32_t* sj = seg + (int64_t)src[u] * (R + 1);
        const int32_t s0 = sj[r], s1 = sj[r_end];
        m_a[i] = row_ptr[src[u]] + s0;
        m_len[i] = s1 - s0;
      }
    }
  }
  __syncthreads();
  const int lo = r * kSegRange;
  const int sub = tid & (kBinGroup - 1);
  constexpr int kGroups = kBinBlock / kBinGroup;
  for (int i = tid / kBinGroup; i < rows; i += kGroups) {
    const int64_t a = m_a[i];
    const int len = m_len[i];
    for (int b0 = 0; b0 < len; b0 += kBinGroup * kBinUnroll) {
      int32_t c[kBinUnroll];
      float wv[kBinUnroll];
#pragma unroll
      for (int u = 0; u < kBinUnroll; ++u) {
        const int k = b0 + u * kBinGroup + sub;
        c[u] = k < len ? col[a + k] : -1;
        wv[u] = k < len ? w[a + k] : 0.0f;
      }
#pragma unroll
      for (int u = 0; u < kBinUnroll; ++u) {
        if (c[u] >= 0) {
          const unsigned long long inc =
              (unsigned long long)__float2ull_rn(fabsf(wv[u]) * scale40);
          atomicAdd(wv[u] > 0.0f ? &se[c[u] - lo] : &si[c[u] - lo], inc);
        }
      }
    }
  }
  __syncthreads();
  for (int t = tid; t < kSpan; t += kBinBlock) {
    const int64_t g = (int64_t)lo + t;
    if (g < n) {
      if (se[t]) atomicAdd(&acc_e[g], se[t]);
      if (si[t]) atomicAdd(&acc_i[g], si[t]);
    }
  }
}

__global__ __launch_bounds__(256) void k_apply(float* __restrict__ ge, float* __restrict__ gi,
                                               unsigned long long* __restrict__ acc_e,
                                               unsigned long long* __restrict__ acc_i, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  ge[i] += (float)acc_e[i] * kUnfix;
  gi[i] += (float)acc_i[i] * kUnfix;
  acc_e[i] = 0ull;
  acc_i[i] = 0ull;
}

// scratch layout: arrival accumulators [2][2][n] (u64), the one-shot
// delivery's list [n], the pull delivery's lists [2][B][N] (i32) and counts
// [3][B] (u32), the one-shot count, the grid barrier's words
size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }
size_t acc_bytes(int64_t n) { return (size_t)4 * n * sizeof(unsigned long long); }
size_t list_off(int64_t n) { return acc_bytes(n); }
size_t plist_off(int64_t n) { return list_off(n) + al256((size_t)n * 4); }
size_t pcount_off(int64_t n) { return plist_off(n) + al256((size_t)n * 8); }
size_t ctr_off(int64_t n, int32_t B) { return pcount_off(n) + al256((size_t)3 * B * 4); }
// grid barrier: the flag-array layout (8 release lines, then one arrival slot
// per block), which also holds the single counter at word 0
size_t bar_words(int64_t n) { return 256 + (size_t)((n + kNetBlock - 1) / kNetBlock); }
size_t bar_off(int64_t n, int32_t B) { return ctr_off(n, B) + 256; }
size_t scratch_size(int64_t n, int32_t B) { return bar_off(n, B) + al256(bar_words(n) * 4); }

template <class S, bool DELAY, bool BATCH, bool PULL, int BS = kNetBlock>
hipError_t launch_net(hh_model* m, NetArgs& a, hipStream_t s) {
  int dev = 0, ncu = 0, per_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_net<S, DELAY, BATCH, PULL, BS>,
                                                   BS, 0);
  if (e != hipSuccess) return e;
  const int64_t nb = (a.n + BS - 1) / BS;
  if (nb > (int64_t)ncu * per_cu) return hipErrorCooperativeLaunchTooLarge;
  hipLaunchKernelGGL(k_net_reset, dim3(1), dim3(256), 0, s, a.bar, (int)bar_words(a.n), a.pcount,
                     3 * a.B);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  void* args[] = {(void*)&m->km, (void*)&a};
  return hipLaunchCooperativeKernel((const void*)k_net<S, DELAY, BATCH, PULL, BS>,
                                    dim3((unsigned)nb), dim3(BS), args, 0, s);
}

}  // namespace

// BS: the block size of the compiled channel sets (the interpreter always
// takes 512-thread blocks)
template <bool DELAY, bool BATCH, bool PULL = false, int BS = kNetBlock>
static hipError_t launch_net_spec(hh_model* m, NetArgs& a, hipStream_t s) {
  if (m->use_fixed && ClassicSpec::matches(m->km))
    return launch_net<ClassicSpec, DELAY, BATCH, PULL, BS>(m, a, s);
  if (m->use_fixed && CorticalSpec::matches(m->km))
    return launch_net<CorticalSpec, DELAY, BATCH, PULL, BS>(m, a, s);
  switch (m->km.n_gates) {
    case 1: return launch_net<GenericSpec<1>, DELAY, BATCH, PULL>(m, a, s);
    case 2: return launch_net<GenericSpec<2>, DELAY, BATCH, PULL>(m, a, s);
    case 3: return launch_net<GenericSpec<3>, DELAY, BATCH, PULL>(m, a, s);
    case 4: return launch_net<GenericSpec<4>, DELAY, BATCH, PULL>(m, a, s);
    case 5: return launch_net<GenericSpec<5>, DELAY, BATCH, PULL>(m, a, s);
    case 6: return launch_net<GenericSpec<6>, DELAY, BATCH, PULL>(m, a, s);
    default: return hipErrorNotSupported;
  }
}

// Delivery by pull with one-step delays when the rows have a segment table
// (and, for a batch, copies of at least one block's 512 elements); by push
// (device atomics into the accumulators) otherwise.
template <bool DELAY>
static hipError_t launch_net_b(hh_model* m, NetArgs& a, hipStream_t s) {
  if constexpr (!DELAY) {
    if (m->d_seg && m->net_pull) {
      // grids of 128 blocks of 512 or more take blocks of 1,024 (half the
      // barrier's arrivals); a batch's copies must then span whole blocks
      const bool wide = (m->n + kNetBlock - 1) / kNetBlock >= kWideMinBlocks &&
                        (m->B == 1 || m->N >= kNetBlockWide);
      if (m->B == 1)
        return wide ? launch_net_spec<false, false, true, kNetBlockWide>(m, a, s)
                    : launch_net_spec<false, false, true>(m, a, s);
      if (m->N >= kNetBlock)
        return wide ? launch_net_spec<false, true, true, kNetBlockWide>(m, a, s)
                    : launch_net_spec<false, true, true>(m, a, s);
    }
  }
  return m->B > 1 ? launch_net_spec<DELAY, true>(m, a, s) : launch_net_spec<DELAY, false>(m, a, s);
}

int32_t hh_net_step_n_internal(hh_model* m, float* state, int64_t t0, int32_t n_steps,
                               const hh_input* in, const hh_outputs* out, void* stream) {
  if (in->mode != HH_IN_NONE && in->mode != HH_IN_CONST && in->mode != HH_IN_BACKGROUND)
    return HH_E_UNSUPPORTED;
  if (m->km.n_gates < 1 || m->km.n_gates > 6) return HH_E_UNSUPPORTED;
  if (out->v_rec || out->ckpt || out->level) return HH_E_UNSUPPORTED;
  if (n_steps == 0) return HH_OK;
  NetArgs a;
  memset(&a, 0, sizeof(a));
  a.state = state;
  a.n = m->n;
  a.N = m->N;
  a.row_ptr = m->row_ptr;
  a.col = m->col;
  a.w = m->w;
  a.w_scale = m->w_scale;
  a.ext_mask = m->ext_mask;
  a.ext_thresh = m->ext_thresh;
  a.w_ext = m->w_ext;
  a.ext_seed = m->ext_seed;
  a.i_const = (in->mode == HH_IN_CONST) ? in->i_const : nullptr;
  if (in->mode == HH_IN_BACKGROUND) {
    a.bg = 1;
    a.mu = in->mu;
    a.sigma = in->sigma;
    a.seed = in->seed;
    a.bg_lam = in->lam;
    a.bg_p0 = (float)exp(-(double)in->lam);
    a.bg_kmax = (int32_t)floor((double)in->lam + 12.0 * sqrt((double)in->lam)) + 12;
  }
  a.t0 = t0;
  a.nsteps = n_steps;
  a.spikes = out->spikes;
  a.words = (m->n + 31) / 32;
  char* sc = (char*)m->d_scratch;
  a.acc = (unsigned long long*)sc;
  a.B = m->B;
  a.bar = (unsigned*)(sc + bar_off(m->n, m->B));
  a.plist = (int32_t*)(sc + plist_off(m->n));
  a.pcount = (unsigned*)(sc + pcount_off(m->n));
  a.seg = m->d_seg;
  a.seg_R = m->seg_R;
  a.flags = m->d_flags;
  a.spin_limit = 1u << 24;
  hipError_t e;
  hipStream_t s = (hipStream_t)stream;
  if (m->delay) {
    a.acc = m->d_ring;
    a.delay = m->delay;
    a.R = m->max_delay + 1;
    if (t0 == 0) {  // a run from the start has nothing in flight
      const int64_t count = (int64_t)a.R * 2 * m->n;
      hipLaunchKernelGGL(k_zero64, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s,
                         m->d_ring, count);
      if ((e = hipGetLastError()) != hipSuccess) return HH_E_HIP;
    }
    e = launch_net_b<true>(m, a, s);
  } else {
    e = launch_net_b<false>(m, a, s);
  }
  if (e == hipErrorCooperativeLaunchTooLarge || e == hipErrorNotSupported) return HH_E_UNSUPPORTED;
  return e == hipSuccess ? HH_OK : HH_E_HIP;
}

extern "C" {

int32_t hh_attach_csr(hh_model* m, const int64_t* row_ptr, const int32_t* col, const float* w,
                      int64_t nnz, float w_scale) {
  if (!m || !row_ptr || (nnz > 0 && (!col || !w))) return HH_E_INVALID;
  if (!m->km.has_syn) return HH_E_INVALID;
  if (nnz < 0) return HH_E_SHAPE;
  if (!(w_scale >= 0.0f) || !std::isfinite(w_scale)) return HH_E_INVALID;
  if (!m->d_scratch) {
    const size_t bytes = scratch_size(m->n, m->B);
    if (hipMalloc(&m->d_scratch, bytes) != hipSuccess) {
      m->d_scratch = nullptr;
      return HH_E_OOM;
    }
    if (hipMemset(m->d_scratch, 0, bytes) != hipSuccess) {
      (void)hipFree(m->d_scratch);  // the next call allocates and clears it again
      m->d_scratch = nullptr;
      return HH_E_HIP;
    }
    m->scratch_bytes = bytes;
  }
  // Every row is read once on the device: the CSR is checked (a bad column
  // or row pointer would send the delivery's writes out of bounds) and, for
  // rows sorted by target, the segment table of the deliveries by target
  // range is built.  The table holds N (R + 1) offsets and is built only
  // while that is no more than the column array (N^2 / 512 grows past it).
  // The device is synchronized first, so the CSR is complete whichever
  // stream wrote it.
  if (hipDeviceSynchronize() != hipSuccess) return HH_E_HIP;
  const int64_t N = m->N;
  const int R = (int)((N + kSegRange - 1) / kSegRange);
  int32_t* seg = nullptr;
  int* flag = nullptr;
  if (nnz > 0 && N * (int64_t)(R + 1) <= nnz &&
      hipMalloc((void**)&seg, (size_t)N * (R + 1) * sizeof(int32_t)) != hipSuccess)
    seg = nullptr;  // no table: the per-event deliveries serve
  if (hipMalloc((void**)&flag, sizeof(int)) != hipSuccess) {
    if (seg) (void)hipFree(seg);
    return HH_E_OOM;
  }
  int flags = 2;
  bool ok = hipMemset(flag, 0, sizeof(int)) == hipSuccess;
  if (ok) {
    hipLaunchKernelGGL(k_csr_segments, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, 0, row_ptr,
                       col, N, nnz, R, seg, flag);
    ok = hipGetLastError() == hipSuccess &&
         hipMemcpy(&flags, flag, sizeof(int), hipMemcpyDeviceToHost) == hipSuccess;
  }
  (void)hipFree(flag);
  if (!ok || (flags & 2)) {
    if (seg) (void)hipFree(seg);
    return ok ? HH_E_INVALID : HH_E_HIP;
  }
  if (flags & 1) {  // unsorted rows: no table
    if (seg) (void)hipFree(seg);
    seg = nullptr;
  }
  // a delay table belongs to the connectivity it was set for
  if (m->d_ring) (void)hipFree(m->d_ring);
  m->d_ring = nullptr;
  m->delay = nullptr;
  m->max_delay = 0;
  m->row_ptr = row_ptr;
  m->col = col;
  m->w = w;
  m->nnz = nnz;
  m->w_scale = w_scale;
  if (m->d_seg) (void)hipFree(m->d_seg);
  m->d_seg = seg;
  m->seg_R = seg ? R : 0;
  return HH_OK;
}

int32_t hh_set_delivery(hh_model* m, int32_t mode) {
  if (!m || (mode != HH_DELIVERY_AUTO && mode != HH_DELIVERY_PUSH)) return HH_E_INVALID;
  m->net_pull = mode == HH_DELIVERY_AUTO ? 1 : 0;
  return HH_OK;
}

int32_t hh_set_external(hh_model* m, const uint8_t* ext_mask, uint32_t thresh, float w_ext,
                        uint64_t seed) {
  if (!m || !std::isfinite(w_ext)) return HH_E_INVALID;
  m->ext_mask = ext_mask;
  m->ext_thresh = thresh;
  m->w_ext = w_ext;
  m->ext_seed = seed;
  return HH_OK;
}

int32_t hh_set_delays(hh_model* m, const uint8_t* delay, int32_t max_delay) {
  if (!m) return HH_E_INVALID;
  if (!delay) {
    if (m->d_ring) (void)hipFree(m->d_ring);
    m->d_ring = nullptr;
    m->delay = nullptr;
    m->max_delay = 0;
    return HH_OK;
  }
  if (!m->row_ptr) return HH_E_INVALID;
  if (max_delay < 1 || max_delay > 255) return HH_E_SHAPE;
  // every delay in [1, max_delay]: checked once here (the kernel also clamps)
  if (m->nnz > 0) {
    uint8_t* h = (uint8_t*)malloc((size_t)m->nnz);
    if (!h) return HH_E_OOM;
    if (hipMemcpy(h, delay, (size_t)m->nnz, hipMemcpyDeviceToHost) != hipSuccess) {
      free(h);
      return HH_E_HIP;
    }
    int bad = 0;
    for (int64_t q = 0; q < m->nnz; ++q) bad |= (h[q] < 1 || h[q] > max_delay);
    free(h);
    if (bad) return HH_E_INVALID;
  }
  const size_t bytes = (size_t)(max_delay + 1) * 2 * (size_t)m->n * sizeof(unsigned long long);
  if (m->d_ring) (void)hipFree(m->d_ring);
  m->d_ring = nullptr;
  if (hipMalloc((void**)&m->d_ring, bytes) != hipSuccess) {
    m->d_ring = nullptr;
    return HH_E_OOM;
  }
  if (hipMemset(m->d_ring, 0, bytes) != hipSuccess) return HH_E_HIP;
  m->delay = delay;
  m->max_delay = max_delay;
  return HH_OK;
}

int32_t hh_syn_propagate(hh_model* m, const uint32_t* spike_bits, float* state,
                         int32_t* n_spikes_out, void* stream) {
  if (!m || !spike_bits || !state) return HH_E_INVALID;
  if (!m->row_ptr || !m->d_scratch) return HH_E_INVALID;
  hipStream_t s = (hipStream_t)stream;
  const int64_t n = m->n;
  char* sc = (char*)m->d_scratch;
  // the one-shot path uses accumulator buffer 1 (the time loop starts on 0
  // and leaves both buffers cleared)
  unsigned long long* acc_e = (unsigned long long*)sc + 2 * n;
  unsigned long long* acc_i = acc_e + n;
  int32_t* list = (int32_t*)(sc + list_off(n));
  unsigned* count = (unsigned*)(sc + ctr_off(n, m->B));
  const int G = m->km.n_gates;
  float* ge = state + (int64_t)(1 + G) * n;
  float* gi = state + (int64_t)(2 + G) * n;
  const unsigned nb = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, count, 1);
  hipLaunchKernelGGL(k_compact, dim3(nb), dim3(256), 0, s, spike_bits, n, list, count);
  int dev = 0, ncu = 256;
  if (hipGetDevice(&dev) == hipSuccess)
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (m->d_seg && m->B == 1) {
    const unsigned chunks = (unsigned)((n + kSegChunk - 1) / kSegChunk);
    const unsigned spans = (unsigned)((m->seg_R + kBinSpan - 1) / kBinSpan);
    hipLaunchKernelGGL(k_scatter_binned, dim3(spans * chunks), dim3(kBinBlock), 0, s, list,
                       count, m->row_ptr, m->col, m->w, m->d_seg, m->seg_R, m->w_scale * kFix,
                       acc_e, acc_i, n);
  } else {
    hipLaunchKernelGGL(k_scatter, dim3((unsigned)ncu * 8), dim3(256), 0, s, list, count, (int)m->N,
                       m->row_ptr, m->col, m->w, m->w_scale * kFix, acc_e, acc_i);
  }
  hipLaunchKernelGGL(k_apply, dim3(nb), dim3(256), 0, s, ge, gi, acc_e, acc_i, n);
  if (n_spikes_out)
    if (hipMemcpyAsync(n_spikes_out, count, sizeof(int32_t), hipMemcpyDeviceToDevice, s) !=
        hipSuccess)
      return HH_E_HIP;
  return hipGetLastError() == hipSuccess ? HH_OK : HH_E_HIP;
}

}
