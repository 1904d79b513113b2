// hh_step.hip -- fused multi-step kernel for independent HH neurons.
//
// One lane owns one neuron.  A launch loads the neuron's V, gates and rate
// coefficients once, runs K steps in registers (operator fusion, Methods
// "Engineering optimization") and stores the state once.  Per step it only
// touches memory for what the caller asked to record: one 64-bit spike word
// per wavefront (ballot), optional V trace, optional checkpoints, and dense
// input current when the current comes from a preceding layer.
#include "hh_internal.h"

using namespace hhk;

template <class S>
__global__ __launch_bounds__(256) void k_init_state(KModel M, float* __restrict__ state, int64_t n,
                                                    int64_t N, const float* __restrict__ coef,
                                                    const float* __restrict__ v0, float v0s) {
  constexpr int NG = S::kNG;
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  LaneRates<NG> L;
  load_rates<S>(M, coef, i % N, N, L);
  const float V = v0 ? v0[i] : v0s;
  state[i] = V;
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    const float r0 = rate_eval<false>(S::form(M, g, 0), L.r[g][0], V, nullptr);
    const float r1 = rate_eval<false>(S::form(M, g, 1), L.r[g][1], V, nullptr);
    state[(int64_t)(1 + g) * n + i] = (S::kind(M, g) == KIND_AB) ? r0 / (r0 + r1) : r0;
  }
  if (M.has_syn) {
    state[(int64_t)(1 + NG) * n + i] = 0.0f;
    state[(int64_t)(2 + NG) * n + i] = 0.0f;
  }
  state[(int64_t)(1 + NG + 2 * M.has_syn) * n + i] = 0.0f;  // low part of V
}

// Time-loop variants.  LOOP_GEN: one step per iteration, any input mode.
// LOOP_DENSE: dense input whose rows are prefetched four steps ahead (the
// loop is unrolled by four so the prefetched values stay in registers).
// LOOP_NOISE: noise input; the four normals of one Philox block feed four
// unrolled steps, so nothing is shuffled between registers from step to step.
// The last two serve the built-in channel sets, where a step is short enough
// that load latency and register copies would otherwise show.
// SYN = false: the population is known to have no synapses, and the synaptic
// terms drop out of the step (bit-identical results).
// LOOP_SINE: sinusoidal input, four steps per iteration like the noise
// loop, the phase carried in a register.
enum { LOOP_GEN = 0, LOOP_DENSE = 1, LOOP_NOISE = 2, LOOP_SINE = 3 };

// TAB: tabulated gate kinetics (A.tab) in place of the rate functions; only
// with uniform coefficients (JIT = false).  TAB_GLOBAL gathers the entries
// from the device table (served by L1/L2); TAB_LDS first copies the table
// into LDS (dynamic size n_gates x n_nodes x 16 bytes), whose bandwidth is
// twice that of the L1 path.
enum { TAB_NONE = 0, TAB_GLOBAL = 1, TAB_LDS = 2 };
// Largest table staged in LDS: the 64 KiB a block may allocate.
constexpr int kTabLdsMaxBytes = 64 * 1024;
// Above this size fewer than six 256-lane blocks share the 160 KB of LDS of a
// compute unit, so large populations take 512-lane blocks: each copy of the
// table then serves eight wavefronts instead of four (a 51 KB table, 641
// nodes of the cortical set: 10.7 against 13.5 ms for 1M x 4,000, the speed
// of a 161-node table).
constexpr int kTabLdsWideBytes = 24 * 1024;

template <class S, bool JIT, int LOOP, bool SYN, int TAB = TAB_NONE>
__global__ __launch_bounds__(TAB == TAB_LDS ? 512 : 256) void k_step(KModel M, StepArgs A) {
  static_assert(!(TAB != TAB_NONE && JIT), "tabulated kinetics need uniform coefficients");
  constexpr bool PF = LOOP == LOOP_DENSE;
  constexpr int NG = S::kNG;
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const bool act = i < A.n;
  const int64_t ii = act ? i : A.n - 1;  // ragged tail: compute on a valid copy, store nothing
  const int64_t n = A.n;
  const int64_t pidx = ii % A.N;

  LaneRates<NG> L;
  load_rates<S>(M, JIT ? A.coef : nullptr, pidx, A.N, L);
  TabRates LT;
  if constexpr (TAB != TAB_NONE) {
    LT.tab = A.tab;
    LT.n = A.tab_n;
    LT.v_lo = A.tab_vlo;
    LT.inv_h = A.tab_inv_h;
  }
  if constexpr (TAB == TAB_LDS) {
    // every lane of the block reaches this point (no early exit above)
    extern __shared__ float4 tab_lds[];
    const int cnt = NG * A.tab_n;
    for (int x = threadIdx.x; x < cnt; x += blockDim.x) tab_lds[x] = A.tab[x];
    __syncthreads();
    LT.tab = tab_lds;
  }
  if constexpr (!JIT && TAB == TAB_NONE && LOOP != LOOP_GEN) {
    // uniform rate offsets pinned in vector registers for the launch, so
    // that x = V s + o reads one scalar operand (s) and needs no copy
#pragma unroll
    for (int g = 0; g < NG; ++g)
#pragma unroll
      for (int r = 0; r < 2; ++r) L.r[g][r].o = pin_vgpr(L.r[g][r].o);
  }
  const float dtC = A.cm ? M.dt / A.cm[pidx] : M.dt / M.C;

  const int64_t row_lo = (int64_t)(1 + NG + 2 * M.has_syn) * n;  // low part of V
  float vh = A.state[ii], vl = A.state[row_lo + ii];
  float p[ng1<NG>];
#pragma unroll
  for (int g = 0; g < NG; ++g) p[g] = A.state[(int64_t)(1 + g) * n + ii];
  float ge = 0.0f, gi = 0.0f;
  if (SYN && M.has_syn) {
    ge = A.state[(int64_t)(1 + NG) * n + ii];
    gi = A.state[(int64_t)(2 + NG) * n + ii];
  }

  // noise: one Philox block gives the normals of four consecutive steps
  float z[4] = {0.f, 0.f, 0.f, 0.f};
  const uint32_t nid = (uint32_t)ii;
  if (A.in_mode == IN_NOISE && (A.t0 & 3)) {
    normals4(A.seed, nid, (uint64_t)A.t0 >> 2, z);
    for (int s = 0; s < (int)(A.t0 & 3); ++s) {
      z[0] = z[1]; z[1] = z[2]; z[2] = z[3];
    }
  }
  const int lane = threadIdx.x & 63;
  const int64_t w0 = (i - lane) >> 5;  // first spike word of this wavefront
  int lvl = 0;
  if constexpr (PF) {
    // dense input: the rows of the next four steps are loaded while the
    // current four are integrated, so no step waits for HBM
    const float* drow = A.i_dense + ii;
    // steps until the next checkpoint (a counter, not a division per step)
    int to_ck = A.ckpt ? (A.ckpt_every - A.k_base % A.ckpt_every) % A.ckpt_every : -1;
    to_ck = __builtin_amdgcn_readfirstlane(to_ck);  // uniform: a scalar register
    float Icur[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (j < A.nsteps) Icur[j] = drow[(int64_t)j * n];
    for (int k0 = 0; k0 < A.nsteps; k0 += 4) {
      float Inext[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (k0 + 4 + j < A.nsteps) Inext[j] = drow[(int64_t)(k0 + 4 + j) * n];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int k = k0 + j;
        if (k >= A.nsteps) break;
        const int kk = A.k_base + k;
        to_ck = __builtin_amdgcn_readfirstlane(to_ck);
        if (to_ck == 0) {
          to_ck = A.ckpt_every;
          if (act) {
            float* c = A.ckpt + (int64_t)(kk / A.ckpt_every) * (2 + NG + 2 * M.has_syn) * n;
            c[i] = vh;
            c[row_lo + i] = vl;
#pragma unroll
            for (int g = 0; g < NG; ++g) c[(int64_t)(1 + g) * n + i] = p[g];
            if (M.has_syn) {
              c[(int64_t)(1 + NG) * n + i] = ge;
              c[(int64_t)(2 + NG) * n + i] = gi;
            }
          }
        }
        if (to_ck > 0) --to_ck;
        const float V = vh;
        if constexpr (TAB != TAB_NONE)
          neuron_step<S, SYN>(M, LT, dtC, vh, vl, p, Icur[j], ge, gi);
        else
          neuron_step<S, SYN>(M, L, dtC, vh, vl, p, Icur[j], ge, gi);
        const float Vn = vh;
        const bool spk = act && (V < M.v_th) && (Vn >= M.v_th);
        if (A.spikes) {
          const uint64_t b = __ballot(spk);
          if (lane == 0 && w0 < A.words) {
            uint32_t* row = A.spikes + (int64_t)k * A.words;
            row[w0] = (uint32_t)b;
            if (w0 + 1 < A.words) row[w0 + 1] = (uint32_t)(b >> 32);
          }
        }
        if (A.v_rec && act) A.v_rec[(int64_t)k * n + i] = Vn;
        lvl += (Vn >= M.v_th);
        if (SYN) {
          ge *= M.decay_e;
          gi *= M.decay_i;
        }
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) Icur[j] = Inext[j];
    }
  } else if constexpr (LOOP == LOOP_NOISE || LOOP == LOOP_SINE) {
    // steps until the next checkpoint (a counter, not a division per step)
    int to_ck = A.ckpt ? (A.ckpt_every - A.k_base % A.ckpt_every) % A.ckpt_every : -1;
    to_ck = __builtin_amdgcn_readfirstlane(to_ck);  // uniform: a scalar register
    auto one_step = [&](int k, float I) {
      to_ck = __builtin_amdgcn_readfirstlane(to_ck);
      if (to_ck == 0) {
        to_ck = A.ckpt_every;
        if (act) {
          float* c = A.ckpt + (int64_t)((A.k_base + k) / A.ckpt_every) * (2 + NG + 2 * M.has_syn) * n;
          c[i] = vh;
          c[row_lo + i] = vl;
#pragma unroll
          for (int g = 0; g < NG; ++g) c[(int64_t)(1 + g) * n + i] = p[g];
          if (M.has_syn) {
            c[(int64_t)(1 + NG) * n + i] = ge;
            c[(int64_t)(2 + NG) * n + i] = gi;
          }
        }
      }
      if (to_ck > 0) --to_ck;
      const float V = vh;
      if constexpr (TAB != TAB_NONE)
        neuron_step<S, SYN>(M, LT, dtC, vh, vl, p, I, ge, gi);
      else
        neuron_step<S, SYN>(M, L, dtC, vh, vl, p, I, ge, gi);
      const float Vn = vh;
      const bool spk = act && (V < M.v_th) && (Vn >= M.v_th);
      if (A.spikes) {
        const uint64_t b = __ballot(spk);
        if (lane == 0 && w0 < A.words) {
          uint32_t* row = A.spikes + (int64_t)k * A.words;
          row[w0] = (uint32_t)b;
          if (w0 + 1 < A.words) row[w0 + 1] = (uint32_t)(b >> 32);
        }
      }
      if (A.v_rec && act) A.v_rec[(int64_t)k * n + i] = Vn;
      lvl += (Vn >= M.v_th);
      if (SYN) {
        ge *= M.decay_e;
        gi *= M.decay_i;
      }
    };
    if constexpr (LOOP == LOOP_SINE) {
      const float amp = A.i_const[ii];
      const uint32_t R = sine_rate(A.freq[ii], A.sine_K);
      uint32_t ph = R * (uint32_t)A.t0;  // R t mod 2^32, advanced by R per step
      for (int k = 0; k < A.nsteps; k += 4) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          if (k + j >= A.nsteps) break;
          one_step(k + j, sine_input(amp, ph));
          ph += R;
        }
      }
    } else {
      // finish the Philox block that an earlier launch began (z was filled
      // and advanced above), then whole blocks of four steps
      const int head = min(A.nsteps, (int)((4 - (A.t0 & 3)) & 3));
      int k = 0;
      for (; k < head; ++k) {
        one_step(k, fmaf(A.sigma, z[0], A.mu));
        z[0] = z[1]; z[1] = z[2]; z[2] = z[3];
      }
      for (; k < A.nsteps; k += 4) {
        normals4(A.seed, nid, (uint64_t)(A.t0 + k) >> 2, z);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          if (k + j >= A.nsteps) break;
          one_step(k + j, fmaf(A.sigma, z[j], A.mu));
        }
      }
    }
  } else {
    // sinusoidal input: amplitude and quantized rate, once per launch
    const float sine_amp = A.in_mode == IN_SINE ? A.i_const[ii] : 0.0f;
    const uint32_t sine_R = A.in_mode == IN_SINE ? sine_rate(A.freq[ii], A.sine_K) : 0u;
    uint32_t sine_ph = sine_R * (uint32_t)A.t0;  // R t mod 2^32, advanced by R per step
    for (int k = 0; k < A.nsteps; ++k) {
      const int64_t t = A.t0 + k;
      const int kk = A.k_base + k;
      if (A.ckpt && (kk % A.ckpt_every) == 0 && act) {
        float* c = A.ckpt + (int64_t)(kk / A.ckpt_every) * (2 + NG + 2 * M.has_syn) * n;
        c[i] = vh;
        c[row_lo + i] = vl;
#pragma unroll
        for (int g = 0; g < NG; ++g) c[(int64_t)(1 + g) * n + i] = p[g];
        if (M.has_syn) {
          c[(int64_t)(1 + NG) * n + i] = ge;
          c[(int64_t)(2 + NG) * n + i] = gi;
        }
      }
      float I = 0.0f;
      if (A.in_mode == IN_CONST) {
        I = A.i_const[ii];
      } else if (A.in_mode == IN_NOISE) {
        if ((t & 3) == 0) normals4(A.seed, nid, (uint64_t)t >> 2, z);
        I = fmaf(A.sigma, z[0], A.mu);
        z[0] = z[1]; z[1] = z[2]; z[2] = z[3];
      } else if (A.in_mode == IN_DENSE) {
        I = A.i_dense[(int64_t)k * n + ii];
      } else if (A.in_mode == IN_BACKGROUND) {
        I = background_current(A.seed, nid, (uint64_t)t, A.bg_lam, A.bg_p0, A.bg_kmax, A.mu,
                               A.sigma);
      } else if (A.in_mode == IN_SINE) {
        I = sine_input(sine_amp, sine_ph);
        sine_ph += sine_R;
      }
      const float V = vh;
      if constexpr (TAB != TAB_NONE)
        neuron_step<S, SYN>(M, LT, dtC, vh, vl, p, I, ge, gi);
      else
        neuron_step<S, SYN>(M, L, dtC, vh, vl, p, I, ge, gi);
      const float Vn = vh;
      const bool spk = act && (V < M.v_th) && (Vn >= M.v_th);
      if (A.spikes) {
        const uint64_t b = __ballot(spk);
        if (lane == 0 && w0 < A.words) {
          uint32_t* row = A.spikes + (int64_t)k * A.words;
          row[w0] = (uint32_t)b;
          if (w0 + 1 < A.words) row[w0 + 1] = (uint32_t)(b >> 32);
        }
      }
      if (A.v_rec && act) A.v_rec[(int64_t)k * n + i] = Vn;
      lvl += (Vn >= M.v_th);
      if constexpr (SYN) {
        ge *= M.decay_e;
        gi *= M.decay_i;
      }
    }
  }

  if (!act) return;
  A.state[i] = vh;
  A.state[row_lo + i] = vl;
  float chk = vh + vl;
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    A.state[(int64_t)(1 + g) * n + i] = p[g];
    chk += p[g];
  }
  if (M.has_syn) {
    A.state[(int64_t)(1 + NG) * n + i] = ge;
    A.state[(int64_t)(2 + NG) * n + i] = gi;
  }
  if (A.level) A.level[i] += (float)lvl;
  if (!__builtin_isfinite(chk)) atomicMin(A.bad, (int32_t)i);
}

// Table of the gate kinetics at nodes V_i = v_lo + i h (one lane per gate and
// node): P = p_inf and Q = 1 - e = -expm1(-dt (alpha + beta)) (or dt / tau),
// evaluated in binary64 from the descriptor's coefficients and rounded once
// per entry, so the nodes carry no error of the step's binary32 rate
// arithmetic (node errors act coherently on every visit of the interval).
struct TabDesc {
  int32_t n_gates;
  int32_t kind[kMaxGates];
  int32_t form[kMaxGates][2];
  double A[kMaxGates][2], B[kMaxGates][2], K[kMaxGates][2], c[kMaxGates][2];
  double dt;
};

__device__ double rate64(int form, double A, double B, double K, double c, double V) {
  const double u = (V - B) / K;
  switch (form) {
    case FORM_EXP: return A * exp(u);
    case FORM_SIGMOID: return A / (1.0 + exp(u));
    case FORM_LINOID: {
      // A (V - B) / (1 - e^{-u}) = A K u / (-expm1(-u)); value A K at u = 0
      const double g = fabs(u) < 1e-12 ? 1.0 + 0.5 * u : u / -expm1(-u);
      return A * K * g;
    }
    default: return (c * exp(u) + exp(-u)) / A;  // FORM_BELL
  }
}

__global__ __launch_bounds__(256) void k_build_table(TabDesc D, double v_lo, double h, int n,
                                                     float4* __restrict__ tab) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= D.n_gates * n) return;
  const int g = x / n, i = x % n;
  double P[2], Q[2];
  for (int j = 0; j < 2; ++j) {
    const double V = v_lo + (double)min(i + j, n - 1) * h;
    const double r0 = rate64(D.form[g][0], D.A[g][0], D.B[g][0], D.K[g][0], D.c[g][0], V);
    const double r1 = rate64(D.form[g][1], D.A[g][1], D.B[g][1], D.K[g][1], D.c[g][1], V);
    const bool ab = D.kind[g] == KIND_AB;
    const double s = ab ? r0 + r1 : r1;  // alpha + beta, or 1 / tau
    P[j] = ab ? r0 / s : r0;
    Q[j] = -expm1(-D.dt * s);
  }
  tab[x] = make_float4((float)P[0], (float)(P[1] - P[0]), (float)Q[0], (float)(Q[1] - Q[0]));
}

template <class S>
static hipError_t init_spec(const hh_model* m, float* state, const float* v0, float v0s,
                            hipStream_t s) {
  const int bs = 256;
  const int64_t nb = (m->n + bs - 1) / bs;
  hipLaunchKernelGGL(k_init_state<S>, dim3((unsigned)nb), dim3(bs), 0, s, m->km, state, m->n,
                     m->N, m->coef, v0, v0s);
  return hipGetLastError();
}

template <class S, int TAB>
static hipError_t step_tab(const hh_model* m, const StepArgs& a, hipStream_t s, dim3 grid, dim3 block,
                           size_t lds) {
  const bool syn = m->km.has_syn != 0;
  if (a.in_mode == IN_DENSE) {
    if (syn) hipLaunchKernelGGL((k_step<S, false, LOOP_DENSE, true, TAB>), grid, block, lds, s, m->km, a);
    else hipLaunchKernelGGL((k_step<S, false, LOOP_DENSE, false, TAB>), grid, block, lds, s, m->km, a);
  } else if (a.in_mode == IN_NOISE) {
    if (syn) hipLaunchKernelGGL((k_step<S, false, LOOP_NOISE, true, TAB>), grid, block, lds, s, m->km, a);
    else hipLaunchKernelGGL((k_step<S, false, LOOP_NOISE, false, TAB>), grid, block, lds, s, m->km, a);
  } else {
    if (syn) hipLaunchKernelGGL((k_step<S, false, LOOP_GEN, true, TAB>), grid, block, lds, s, m->km, a);
    else hipLaunchKernelGGL((k_step<S, false, LOOP_GEN, false, TAB>), grid, block, lds, s, m->km, a);
  }
  return hipGetLastError();
}

template <class S>
static hipError_t step_spec(const hh_model* m, const StepArgs& a, hipStream_t s) {
  // Small populations use 64-lane blocks so their few wavefronts spread over
  // as many compute units as possible (the step is latency bound there).
  const int bs = (a.n < 65536) ? 64 : 256;
  const dim3 grid((unsigned)((a.n + bs - 1) / bs)), block(bs);
  const bool jit = a.coef != nullptr;
  if constexpr (S::kFixed) {
    const bool syn = m->km.has_syn != 0;
    if (a.tab) {  // validated when the table was set: uniform coefficients
      const size_t bytes = (size_t)S::kNG * (size_t)a.tab_n * sizeof(float4);
      if (bytes > (size_t)kTabLdsWideBytes && bytes <= (size_t)kTabLdsMaxBytes && a.n >= 65536) {
        const dim3 wgrid((unsigned)((a.n + 511) / 512)), wblock(512);
        return step_tab<S, TAB_LDS>(m, a, s, wgrid, wblock, bytes);
      }
      if (bytes <= (size_t)kTabLdsMaxBytes) return step_tab<S, TAB_LDS>(m, a, s, grid, block, bytes);
      return step_tab<S, TAB_GLOBAL>(m, a, s, grid, block, 0);
    }
    if (a.in_mode == IN_DENSE || a.in_mode == IN_NOISE || a.in_mode == IN_SINE) {
#define HH_LAUNCH(LOOP)                                                                        \
  do {                                                                                         \
    if (jit && syn) hipLaunchKernelGGL((k_step<S, true, LOOP, true>), grid, block, 0, s, m->km, a);   \
    else if (jit) hipLaunchKernelGGL((k_step<S, true, LOOP, false>), grid, block, 0, s, m->km, a);    \
    else if (syn) hipLaunchKernelGGL((k_step<S, false, LOOP, true>), grid, block, 0, s, m->km, a);    \
    else hipLaunchKernelGGL((k_step<S, false, LOOP, false>), grid, block, 0, s, m->km, a);            \
  } while (0)
      if (a.in_mode == IN_DENSE) HH_LAUNCH(LOOP_DENSE);
      else if (a.in_mode == IN_SINE) HH_LAUNCH(LOOP_SINE);
      else HH_LAUNCH(LOOP_NOISE);
#undef HH_LAUNCH
      return hipGetLastError();
    }
  }
  // general loop: the synapse-free variant for the compiled channel sets
  // without synapses (bit-identical, fewer operations), the synaptic one
  // otherwise
  if constexpr (S::kFixed) {
    if (!m->km.has_syn) {
      if (jit) hipLaunchKernelGGL((k_step<S, true, LOOP_GEN, false>), grid, block, 0, s, m->km, a);
      else hipLaunchKernelGGL((k_step<S, false, LOOP_GEN, false>), grid, block, 0, s, m->km, a);
      return hipGetLastError();
    }
  }
  if (jit)
    hipLaunchKernelGGL((k_step<S, true, LOOP_GEN, true>), grid, block, 0, s, m->km, a);
  else
    hipLaunchKernelGGL((k_step<S, false, LOOP_GEN, true>), grid, block, 0, s, m->km, a);
  return hipGetLastError();
}

template <class S>
struct InitF {
  static hipError_t run(const hh_model* m, float* state, const float* v0, float v0s, hipStream_t s) {
    return init_spec<S>(m, state, v0, v0s, s);
  }
};
template <class S>
struct StepF {
  static hipError_t run(const hh_model* m, const StepArgs& a, hipStream_t s) {
    return step_spec<S>(m, a, s);
  }
};

hipError_t launch_init_state(const hh_model* m, float* state, const float* v0, float v0s,
                             hipStream_t s) {
  return dispatch_spec<InitF>(m->km, m->use_fixed, m, state, v0, v0s, s);
}

hipError_t launch_step(const hh_model* m, const StepArgs& a, hipStream_t s) {
  return dispatch_spec<StepF, const hh_model*, const StepArgs&, hipStream_t>(m->km, m->use_fixed, m,
                                                                               a, s);
}

hipError_t launch_build_table(const hh_model* m, hipStream_t s) {
  TabDesc D = {};
  const hh_model_desc& d = m->desc;
  D.n_gates = d.n_gates;
  for (int g = 0; g < d.n_gates; ++g) {
    D.kind[g] = d.gates[g].kind;
    for (int r = 0; r < 2; ++r) {
      const hh_rate& q = d.gates[g].r[r];
      D.form[g][r] = q.form;
      D.A[g][r] = q.A;
      D.B[g][r] = q.B;
      D.K[g][r] = q.K;
      D.c[g][r] = q.c;
    }
  }
  D.dt = d.dt;
  const int count = d.n_gates * m->tab_n;
  hipLaunchKernelGGL(k_build_table, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, D,
                     (double)m->tab_vlo, 1.0 / (double)m->tab_inv_h, m->tab_n, m->d_tab);
  return hipGetLastError();
}
