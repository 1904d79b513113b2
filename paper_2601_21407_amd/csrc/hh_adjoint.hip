// hh_adjoint.hip -- backpropagation through time of the discrete HH map
// (Methods, "Gradient learning support"; "Engineering optimization":
// manually derived gradients with re-computation).
//
// One lane owns one neuron and walks its checkpoint segments in reverse.  A
// segment of S steps is replayed from its checkpoint; when S exceeds the
// register window R, a first replay stores the state at every R-th step in
// a workspace.  The first replays of all segments of a call are independent
// of the adjoint and of each other, so they run first, as one kernel over
// (segment, neuron) -- many more wavefronts than the neurons alone give,
// which hides the latency of the step's dependent chain.  Each R-step
// window is then replayed once more, and
// that replay evaluates every step's transposed Jacobian from the same rate
// evaluations that advance the state, keeping only the Jacobian entries in
// registers.  The reverse sweep over the window then only carries the
// adjoint lambda = (lambda_V, lambda_p) through those entries.  They are
// closed form in the rate functions and their V-derivatives:
//   dV'/dV = 1 - (dt/C) g_tot,   dV'/dp_g = -(dt/C) sum_X gbar dEta_X/dp_g (V - E_X)
//   dp'/dp = e,   dp'/dV = p_inf' (1 - e) + (p - p_inf) e'
//   dV'/dI = dt/C,   dV'/dC = -(dt/C^2) (I - I_ion)
// The spike output is the level H(V - v_th); its derivative is replaced by
// the surrogate beta s (1 - s), s = sigmoid(beta (V - v_th)).
#include <string.h>

#include "hh_internal.h"

using namespace hhk;

namespace {

constexpr int kWin = 5;  // register window R

struct BwdArgs {
  const float* ckpt;  // [nseg][ns][n]
  int32_t S, T;
  const float* I;     // [T][n]
  const float* dlevel;
  const float* dV;    // [T][n]
  float beta, inv_T;
  float* dI;          // [T][n]
  float* dC_part;     // [n]
  float* dx0;         // [ns][n]
  float* sub;         // [nseg][ceil(S/R)][ns][n]: window starts of every segment
  float* lam;         // [1 + NG][n]: the adjoint carried between partial calls
  int32_t j_lo, j_hi; // checkpoint segments [j_lo, j_hi) of this call, in reverse
  int32_t first;      // no later segment: lambda and dC start at zero
  int32_t last;       // segment 0 included: write dx0
  int64_t n, N;
  const float* cm;
  const float* coef;
};

// Transposed-Jacobian entries of one step, and the surrogate derivative of
// the level at the step's end state.
template <class S>
struct StepJ {
  float e[ng1<S::kNG>], dpv[ng1<S::kNG>], dvdp[ng1<S::kNG>];
  float dvdv, dvdC, sgd;
};

// One explicit-Euler step without synapses -- the arithmetic of
// neuron_step, in the same order -- that also returns its Jacobian entries.
template <class S>
__device__ __forceinline__ void step_with_jacobian(const KModel& M, const LaneRates<S::kNG>& L,
                                                   float dtC, float C, float& vh, float& vl,
                                                   float (&p)[ng1<S::kNG>], float I, StepJ<S>& J) {
  constexpr int NG = S::kNG;
  const float V = vh;
  const float ndt = M.kdt * kLn2;  // -dt
  // channel terms at the start-of-step gates, and dI_ion/dp_g
  float gsum = 0.0f, esum = 0.0f, b[ng1<NG>];
#pragma unroll
  for (int g = 0; g < NG; ++g) b[g] = 0.0f;
#pragma unroll
  for (int c = 0; c < kMaxCh; ++c) {
    if (c >= S::nch(M)) break;
    float pw[ng1<NG>];
    float eta = M.gbar[c];
#pragma unroll
    for (int g = 0; g < NG; ++g) {
      const int ex = S::cexp(M, c, g);
      pw[g] = ex ? ipow(p[g], ex) : 1.0f;
      if (ex) eta *= pw[g];
    }
    gsum += eta;
    esum = fmaf(eta, M.E[c], esum);
    const float vme = V - M.E[c];
#pragma unroll
    for (int g = 0; g < NG; ++g) {
      const int ex = S::cexp(M, c, g);
      if (ex) {
        float d = M.gbar[c] * (float)ex * ipow(p[g], ex - 1);
#pragma unroll
        for (int g2 = 0; g2 < NG; ++g2)
          if (g2 != g) d *= pw[g2];
        b[g] = fmaf(d, vme, b[g]);
      }
    }
  }
  // gates by exponential Euler at V_t, with dp'/dp and dp'/dV
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    float d0, d1;
    const float r0 = rate_eval<true>(S::form(M, g, 0), L.r[g][0], V, &d0);
    const float r1 = rate_eval<true>(S::form(M, g, 1), L.r[g][1], V, &d1);
    float pinf, dpinf, e, q, de;  // q = 1 - e, formed as the forward step forms it
    if (S::kind(M, g) == KIND_AB) {
      const float sr = r0 + r1, is = rcp(sr);
      pinf = r0 * is;
      dpinf = (d0 * r1 - r0 * d1) * is * is;
      e = ex2(sr * M.kdt);
      q = 1.0f - e;
      de = ndt * (d0 + d1) * e;
    } else {
      pinf = r0;
      dpinf = d0;
      q = one_minus_exp_neg(r1 * M.dt);
      e = 1.0f - q;
      de = ndt * d1 * e;
    }
    J.e[g] = e;
    J.dpv[g] = fmaf(dpinf, q, (p[g] - pinf) * de);
    p[g] = fmaf(pinf - p[g], q, p[g]);
  }
  // membrane (explicit Euler)
  const float iion = fmaf(gsum, vl, fmaf(gsum, V, -esum));
  const float dv = dtC * (I - iion);
  J.dvdv = fmaf(-dtC, gsum, 1.0f);
  J.dvdC = -(dtC / C) * (I - iion);
#pragma unroll
  for (int g = 0; g < NG; ++g) J.dvdp[g] = -dtC * b[g];
  add_to_v(vh, vl, dv);
}

// First replay of segment j = j_lo + blockIdx.y: the state at the start of
// each R-step window of the segment into the workspace (the last window's
// steps are not needed).  The same arithmetic as the forward step.
template <class S>
__global__ __launch_bounds__(256) void k_replay(KModel M, BwdArgs A) {
  constexpr int NG = S::kNG;
  const int64_t n = A.n;
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int j = A.j_lo + (int)blockIdx.y;
  const int ta = j * A.S, tb = min(ta + A.S, A.T);
  const int nwin = (tb - ta + kWin - 1) / kWin;
  if (nwin <= 1) return;
  const int64_t pidx = i % A.N;
  const int ns = 2 + NG;
  const int wmax = (A.S + kWin - 1) / kWin;
  LaneRates<NG> L;
  load_rates<S>(M, A.coef, pidx, A.N, L);
  const float dtC = M.dt / (A.cm ? A.cm[pidx] : M.C);
  const float* ck = A.ckpt + (int64_t)j * ns * n;
  float vh = ck[i], vl = ck[(int64_t)(1 + NG) * n + i], p[ng1<NG>];
#pragma unroll
  for (int g = 0; g < NG; ++g) p[g] = ck[(int64_t)(1 + g) * n + i];
  for (int w = 0; w < nwin; ++w) {
    float* ws = A.sub + ((int64_t)j * wmax + w) * ns * n;
    ws[i] = vh;
    ws[(int64_t)(1 + NG) * n + i] = vl;
#pragma unroll
    for (int g = 0; g < NG; ++g) ws[(int64_t)(1 + g) * n + i] = p[g];
    if (w + 1 == nwin) break;
    const int ua = ta + w * kWin;  // a full window: only the last can be short
    float Icur[kWin];
#pragma unroll
    for (int k = 0; k < kWin; ++k) Icur[k] = A.I[(int64_t)(ua + k) * n + i];
#pragma unroll
    for (int k = 0; k < kWin; ++k) neuron_step<S>(M, L, dtC, vh, vl, p, Icur[k], 0.0f, 0.0f);
  }
}

template <class S>
__global__ __launch_bounds__(256) void k_bptt(KModel M, BwdArgs A) {
  constexpr int NG = S::kNG;
  const int64_t n = A.n;
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;  // lanes are independent: no wave-level operations below
  const int64_t pidx = i % A.N;
  const int ns = 2 + NG;
  LaneRates<NG> L;
  load_rates<S>(M, A.coef, pidx, A.N, L);
  const float C = A.cm ? A.cm[pidx] : M.C;
  const float dtC = M.dt / C;

  // adjoint at the end of this call's range: zero at T, else left by the
  // call for the later segments
  float lamV = 0.0f, lamP[ng1<NG>];
#pragma unroll
  for (int g = 0; g < NG; ++g) lamP[g] = 0.0f;
  float dc = 0.0f;
  if (!A.first) {
    lamV = A.lam[i];
#pragma unroll
    for (int g = 0; g < NG; ++g) lamP[g] = A.lam[(int64_t)(1 + g) * n + i];
    dc = A.dC_part[i];
  }
  // the loss term on the level, per step: dL/dlevel / T
  const float dlv = A.dlevel ? A.dlevel[i] * A.inv_T : 0.0f;

  for (int j = A.j_hi - 1; j >= A.j_lo; --j) {
    const int ta = j * A.S, tb = min(ta + A.S, A.T);
    const float* ck = A.ckpt + (int64_t)j * ns * n;
    const int nwin = (tb - ta + kWin - 1) / kWin;
    // window starts: from k_replay, or the checkpoint itself for one window
    const float* sub_j = A.sub + (int64_t)j * ((A.S + kWin - 1) / kWin) * ns * n;
    for (int q = nwin - 1; q >= 0; --q) {
      const int ua = ta + q * kWin, ub = min(ua + kWin, tb);
      const float* src = (nwin > 1) ? sub_j + (int64_t)q * ns * n : ck;
      float vh = src[i], vl = src[(int64_t)(1 + NG) * n + i], p[ng1<NG>];
#pragma unroll
      for (int g = 0; g < NG; ++g) p[g] = src[(int64_t)(1 + g) * n + i];
      float Iv[kWin];
#pragma unroll
      for (int k = 0; k < kWin; ++k) Iv[k] = ua + k < ub ? A.I[(int64_t)(ua + k) * n + i] : 0.0f;
      // replay the window, keeping each step's Jacobian entries
      StepJ<S> J[kWin];
#pragma unroll
      for (int k = 0; k < kWin; ++k) {
        if (ua + k < ub) {
          step_with_jacobian<S>(M, L, dtC, C, vh, vl, p, Iv[k], J[k]);
          J[k].sgd = 0.0f;
          if (A.dlevel) {
            const float sg = rcp(1.0f + ex2(-A.beta * (vh - M.v_th) * kLog2e));
            J[k].sgd = A.beta * sg * (1.0f - sg);
          }
        }
      }
      // reverse sweep
#pragma unroll
      for (int k = kWin - 1; k >= 0; --k) {
        if (ua + k < ub) {
          const int t = ua + k;
          // direct loss on V_{t+1}
          if (A.dlevel) lamV = fmaf(dlv, J[k].sgd, lamV);
          if (A.dV) lamV += A.dV[(int64_t)t * n + i];
          A.dI[(int64_t)t * n + i] = lamV * dtC;
          dc = fmaf(lamV, J[k].dvdC, dc);
          float nv = lamV * J[k].dvdv;
#pragma unroll
          for (int g = 0; g < NG; ++g) {
            nv = fmaf(lamP[g], J[k].dpv[g], nv);
            lamP[g] = fmaf(lamV, J[k].dvdp[g], lamP[g] * J[k].e[g]);
          }
          lamV = nv;
        }
      }
    }
  }
  A.dC_part[i] = dc;
  if (!A.last) {
    A.lam[i] = lamV;
#pragma unroll
    for (int g = 0; g < NG; ++g) A.lam[(int64_t)(1 + g) * n + i] = lamP[g];
    return;
  }
  if (A.dx0) {
    A.dx0[i] = lamV;
#pragma unroll
    for (int g = 0; g < NG; ++g) A.dx0[(int64_t)(1 + g) * n + i] = lamP[g];
    A.dx0[(int64_t)(1 + NG) * n + i] = lamV;  // V = V + V_lo
  }
}

// dCm[h] = sum over the batch: a block owns 64 units h; its 16 lane groups
// each sum a sixteenth of the batch, and the partial sums are added in group
// order (deterministic).
constexpr int SBH = 64, SBG = 16;

__global__ __launch_bounds__(SBH * SBG) void k_sum_batch(const float* __restrict__ part,
                                                         float* __restrict__ out, int64_t N,
                                                         int32_t B) {
  __shared__ float red[SBG][SBH];
  const int hx = threadIdx.x % SBH, g = threadIdx.x / SBH;
  const int64_t h = blockIdx.x * (int64_t)SBH + hx;
  const int per = (B + SBG - 1) / SBG;
  const int b0 = g * per, b1 = min(B, b0 + per);
  float s = 0.0f;
  if (h < N) {
    // eight loads in flight, added in batch order (the same sum as one at a time)
    int b = b0;
    for (; b + 8 <= b1; b += 8) {
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = part[(int64_t)(b + u) * N + h];
#pragma unroll
      for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; b < b1; ++b) s += part[(int64_t)b * N + h];
  }
  red[g][hx] = s;
  __syncthreads();
  if (g == 0 && h < N) {
    float t = 0.0f;
    for (int q = 0; q < SBG; ++q) t += red[q][hx];
    out[h] = t;
  }
}

template <class S>
hipError_t launch_bptt(const hh_model* m, const BwdArgs& a, hipStream_t s) {
  const int64_t nb = (a.n + 255) / 256;
  if ((a.S + kWin - 1) / kWin > 1) {
    hipLaunchKernelGGL(k_replay<S>, dim3((unsigned)nb, (unsigned)(a.j_hi - a.j_lo)), dim3(256), 0,
                       s, m->km, a);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_bptt<S>, dim3((unsigned)nb), dim3(256), 0, s, m->km, a);
  return hipGetLastError();
}

// window starts of every segment: nseg x ceil(S / R) x (2 + NG) x n floats
size_t sub_bytes(const hh_model* m, int32_t S, int32_t T) {
  const int nwin = (S + kWin - 1) / kWin;
  if (nwin <= 1) return 0;
  const size_t nseg = (size_t)((T + S - 1) / S);
  return nseg * (size_t)nwin * (size_t)(2 + m->km.n_gates) * (size_t)m->n * sizeof(float);
}

}  // namespace

extern "C" {

size_t hh_backward_workspace(const hh_model* m, int32_t ckpt_every, int32_t T) {
  if (!m || ckpt_every < 1 || T < 1) return 0;
  const size_t part = (((size_t)m->n * sizeof(float)) + 255) & ~(size_t)255;
  const size_t lam = ((((size_t)(1 + m->km.n_gates) * m->n * sizeof(float)) + 255) & ~(size_t)255);
  return part + lam + sub_bytes(m, ckpt_every, T);
}

int32_t hh_backward_part(hh_model* m, const float* ckpt, int32_t ckpt_every, const hh_input* in,
                         int32_t T, int32_t t_lo, int32_t t_hi, const float* dL_dlevel,
                         const float* dL_dV, float beta, float* dI, float* dCm, float* dx0,
                         void* workspace, size_t workspace_bytes, void* stream) {
  if (!m || !ckpt || !in || !dI) return HH_E_INVALID;
  if (m->km.has_syn || m->km.v_method != HH_V_FE) return HH_E_UNSUPPORTED;
  if (m->d_tab) return HH_E_UNSUPPORTED;  // the adjoint differentiates the rate functions
  if (m->d_cable) return HH_E_UNSUPPORTED;  // and has no axial coupling
  if (in->mode != HH_IN_DENSE || !in->i_dense) return HH_E_INVALID;
  if (T < 1 || ckpt_every < 1) return HH_E_SHAPE;
  if (t_lo < 0 || t_hi > T || t_lo >= t_hi || t_lo % ckpt_every != 0 ||
      (t_hi != T && t_hi % ckpt_every != 0))
    return HH_E_SHAPE;
  if (!(beta > 0.0f)) return HH_E_INVALID;
  const size_t need = hh_backward_workspace(m, ckpt_every, T);
  if (!workspace || workspace_bytes < need) return HH_E_SHAPE;
  BwdArgs a;
  memset(&a, 0, sizeof(a));
  a.ckpt = ckpt;
  a.S = ckpt_every;
  a.T = T;
  a.I = in->i_dense;
  a.dlevel = dL_dlevel;
  a.dV = dL_dV;
  a.beta = beta;
  a.inv_T = 1.0f / (float)T;
  a.dI = dI;
  const size_t part = (((size_t)m->n * sizeof(float)) + 255) & ~(size_t)255;
  const size_t lam = ((((size_t)(1 + m->km.n_gates) * m->n * sizeof(float)) + 255) & ~(size_t)255);
  a.dC_part = (float*)workspace;
  a.lam = (float*)((char*)workspace + part);
  a.sub = (float*)((char*)workspace + part + lam);
  a.dx0 = dx0;
  a.j_lo = t_lo / ckpt_every;
  a.j_hi = (t_hi + ckpt_every - 1) / ckpt_every;
  a.first = t_hi == T;
  a.last = t_lo == 0;
  a.n = m->n;
  a.N = m->N;
  a.cm = m->cm;
  a.coef = m->coef;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e;
  if (m->use_fixed && ClassicSpec::matches(m->km)) {
    e = launch_bptt<ClassicSpec>(m, a, s);
  } else if (m->use_fixed && CorticalSpec::matches(m->km)) {
    e = launch_bptt<CorticalSpec>(m, a, s);
  } else {
    switch (m->km.n_gates) {
      case 0: e = launch_bptt<GenericSpec<0>>(m, a, s); break;
      case 1: e = launch_bptt<GenericSpec<1>>(m, a, s); break;
      case 2: e = launch_bptt<GenericSpec<2>>(m, a, s); break;
      case 3: e = launch_bptt<GenericSpec<3>>(m, a, s); break;
      case 4: e = launch_bptt<GenericSpec<4>>(m, a, s); break;
      case 5: e = launch_bptt<GenericSpec<5>>(m, a, s); break;
      case 6: e = launch_bptt<GenericSpec<6>>(m, a, s); break;
      default: return HH_E_UNSUPPORTED;
    }
  }
  if (e != hipSuccess) return HH_E_HIP;
  if (dCm && a.last) {
    hipLaunchKernelGGL(k_sum_batch, dim3((unsigned)((m->N + SBH - 1) / SBH)), dim3(SBH * SBG), 0,
                       s, a.dC_part, dCm, m->N, m->B);
    if (hipGetLastError() != hipSuccess) return HH_E_HIP;
  }
  return HH_OK;
}

int32_t hh_backward(hh_model* m, const float* ckpt, int32_t ckpt_every, const hh_input* in,
                    int32_t T, const float* dL_dlevel, const float* dL_dV, float beta, float* dI,
                    float* dCm, float* dx0, void* workspace, size_t workspace_bytes, void* stream) {
  if (T < 1) return HH_E_SHAPE;
  return hh_backward_part(m, ckpt, ckpt_every, in, T, 0, T, dL_dlevel, dL_dV, beta, dI, dCm, dx0,
                          workspace, workspace_bytes, stream);
}

}  // extern "C"
