// hh_cable.hip -- multi-compartment neurons: the spatial term of the cable
// equation (Methods, Eq. (1)) by the second-order explicit difference
// (Methods, "Simplified discretization").
//
// A neuron is K consecutive compartments of the population (K a power of two
// up to 64), so the compartments of one neuron always share a wavefront and
// exchange their potentials with ds_bpermute, without LDS or barriers.  Each
// step, compartment c receives the axial current
//     I_ax = sum over its edges e of (g_e / area_c) (V_other(e) - V_c)
// from the start-of-step potentials (for a uniform cable with
// g = 1 / (r_l dx^2) this is (1/r_l) (V_{c-1} - 2 V_c + V_{c+1}) / dx^2),
// and the neuron step then runs unchanged with I + I_ax as its input.
#include "hh_internal.h"

using namespace hhk;

namespace {

// V of the lane at byte address `addr` within the wavefront
__device__ __forceinline__ float lane_v(int addr, float v) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(v)));
}

// TAB: 0 the rate functions, 1 tabulated kinetics read from device memory,
// 2 the table staged in LDS (as in the point step).
template <class S, bool SYN, bool GBAR, int TAB>
__global__ __launch_bounds__(TAB == 2 ? 512 : 256) void k_cable(KModel M, StepArgs A) {
  constexpr int NG = S::kNG;
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const bool act = i < A.n;
  const int64_t ii = act ? i : A.n - 1;  // ragged tail: compute on a valid copy, store nothing
  const int64_t n = A.n;
  const int64_t pidx = ii % A.N;
  const int lane = threadIdx.x & 63;

  // this lane's compartment: taken from i, not ii, so that idle lanes of the
  // last wavefront still form whole neurons among themselves
  const int K = A.cable_K;
  const int c = (int)(i & (int64_t)(K - 1));
  const CableComp& CC = A.cable[c];
  const int base = lane & ~(K - 1);
  const int a_par = (base + CC.par) * 4;
  int a_ch[kMaxChildren];
  float gdn[kMaxChildren];
#pragma unroll
  for (int d = 0; d < kMaxChildren; ++d) {
    a_ch[d] = (base + CC.ch[d]) * 4;
    gdn[d] = CC.gdn[d];
  }
  const float gup = CC.gup;
  const int D = A.cable_D;
  LaneGbar G;
  if constexpr (GBAR) {
#pragma unroll
    for (int x = 0; x < kMaxCh; ++x) G.g[x] = CC.gbar[x];
  }

  LaneRates<NG> L;
  load_rates<S>(M, A.coef, pidx, A.N, L);
  TabRates LT;
  if constexpr (TAB != 0) {
    LT.tab = A.tab;
    LT.n = A.tab_n;
    LT.v_lo = A.tab_vlo;
    LT.inv_h = A.tab_inv_h;
  }
  if constexpr (TAB == 2) {
    // every lane of the block reaches this point (no early exit above)
    extern __shared__ float4 cable_tab[];
    const int cnt = NG * A.tab_n;
    for (int x = threadIdx.x; x < cnt; x += blockDim.x) cable_tab[x] = A.tab[x];
    __syncthreads();
    LT.tab = cable_tab;
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

  float z[4] = {0.f, 0.f, 0.f, 0.f};
  const uint32_t nid = (uint32_t)ii;
  if (A.in_mode == IN_NOISE && (A.t0 & 3)) {
    normals4(A.seed, nid, (uint64_t)A.t0 >> 2, z);
    for (int s = 0; s < (int)(A.t0 & 3); ++s) {
      z[0] = z[1]; z[1] = z[2]; z[2] = z[3];
    }
  }
  const int64_t w0 = (i - lane) >> 5;  // first spike word of this wavefront

  for (int k = 0; k < A.nsteps; ++k) {
    const int64_t t = A.t0 + k;
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
    }
    // axial current from the start-of-step potentials of the neighbours
    const float V = vh;
    float iax = gup * (lane_v(a_par, V) - V);
#pragma unroll
    for (int d = 0; d < kMaxChildren; ++d)
      if (d < D) iax = fmaf(gdn[d], lane_v(a_ch[d], V) - V, iax);
    if constexpr (TAB != 0 && GBAR)
      neuron_step<S, SYN>(M, LT, dtC, vh, vl, p, I + iax, ge, gi, G);
    else if constexpr (TAB != 0)
      neuron_step<S, SYN>(M, LT, dtC, vh, vl, p, I + iax, ge, gi);
    else if constexpr (GBAR)
      neuron_step<S, SYN>(M, L, dtC, vh, vl, p, I + iax, ge, gi, G);
    else
      neuron_step<S, SYN>(M, L, dtC, vh, vl, p, I + iax, ge, gi);
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
    if constexpr (SYN) {
      ge *= M.decay_e;
      gi *= M.decay_i;
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
  if (SYN && M.has_syn) {
    A.state[(int64_t)(1 + NG) * n + i] = ge;
    A.state[(int64_t)(2 + NG) * n + i] = gi;
  }
  if (!__builtin_isfinite(chk)) atomicMin(A.bad, (int32_t)i);
}

template <class S, int TAB>
static hipError_t launch_cable_tab(const hh_model* m, const StepArgs& a, hipStream_t s, dim3 grid,
                                   dim3 block, size_t lds) {
  const bool syn = m->km.has_syn != 0;
  if (m->cable_gbar) {
    if (syn) hipLaunchKernelGGL((k_cable<S, true, true, TAB>), grid, block, lds, s, m->km, a);
    else hipLaunchKernelGGL((k_cable<S, false, true, TAB>), grid, block, lds, s, m->km, a);
  } else {
    if (syn) hipLaunchKernelGGL((k_cable<S, true, false, TAB>), grid, block, lds, s, m->km, a);
    else hipLaunchKernelGGL((k_cable<S, false, false, TAB>), grid, block, lds, s, m->km, a);
  }
  return hipGetLastError();
}

// Largest table staged in LDS: the 64 KiB a block may allocate.  Above 24 KiB
// large populations take 512-lane blocks, so that each copy of the table
// serves eight wavefronts (blocks of whole wavefronts never split a neuron).
constexpr int kCableTabLdsMaxBytes = 64 * 1024;
constexpr int kCableTabLdsWideBytes = 24 * 1024;

template <class S>
struct CableF {
  static hipError_t run(const hh_model* m, const StepArgs& a, hipStream_t s) {
    // 64-lane blocks for small populations spread them over more compute units
    const int bs = (a.n < 65536) ? 64 : 256;
    const dim3 grid((unsigned)((a.n + bs - 1) / bs)), block(bs);
    if constexpr (S::kFixed) {
      if (a.tab) {  // tables exist for the compiled channel sets only
        const size_t bytes = (size_t)S::kNG * (size_t)a.tab_n * sizeof(float4);
        if (bytes > (size_t)kCableTabLdsWideBytes && bytes <= (size_t)kCableTabLdsMaxBytes &&
            a.n >= 65536) {
          const dim3 wgrid((unsigned)((a.n + 511) / 512)), wblock(512);
          return launch_cable_tab<S, 2>(m, a, s, wgrid, wblock, bytes);
        }
        if (bytes <= (size_t)kCableTabLdsMaxBytes) return launch_cable_tab<S, 2>(m, a, s, grid, block, bytes);
        return launch_cable_tab<S, 1>(m, a, s, grid, block, 0);
      }
    }
    return launch_cable_tab<S, 0>(m, a, s, grid, block, 0);
  }
};

}  // namespace

hipError_t launch_cable(const hh_model* m, const StepArgs& a, hipStream_t s) {
  return dispatch_spec<CableF, const hh_model*, const StepArgs&, hipStream_t>(m->km, m->use_fixed,
                                                                                m, a, s);
}
