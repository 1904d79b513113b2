// hh_device.h -- device-side building blocks of the HH hot path for gfx950.
//
// Per-neuron arithmetic of one time step (Methods, Eq. (1)-(2), "Simplified
// discretization"): rate functions, exponential-Euler gates, channel currents,
// the membrane update and threshold crossing.  Everything here is evaluated
// in FP32 registers; transcendental functions go straight to the CDNA
// special-function unit (v_exp_f32 = 2^x, v_log_f32 = log2, v_rcp_f32,
// v_sqrt_f32, v_sin_f32/v_cos_f32 taking their argument in revolutions).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hhk {

constexpr int kMaxGates = 8;
constexpr int kMaxCh = 8;
constexpr float kLog2e = 1.4426950408889634f;
constexpr float kLn2 = 0.6931471805599453f;

enum { FORM_EXP = 0, FORM_SIGMOID = 1, FORM_LINOID = 2, FORM_BELL = 3 };
enum { KIND_AB = 0, KIND_INFTAU = 1 };
enum { VFE = 0, VEE = 1 };
enum { IN_NONE = 0, IN_CONST = 1, IN_NOISE = 2, IN_DENSE = 3, IN_BACKGROUND = 4, IN_SINE = 5 };

// One rate function in a form ready for the exp2 unit.  With x = V*s + o =
// log2(e) (V - B) / K:
//   exp      r = a 2^x                       a = A
//   sigmoid  r = a / (1 + 2^x)               a = A
//   linoid   r = a g(u), u = x ln2,          a = A K,  g(u) = u / (1 - e^{-u})
//   bell     r = a (c 2^x + 2^-x)            a = 1 / A
// ik = 1/K scales the V-derivatives.
struct KRate {
  float s, o, a, c, ik;
};

// Kernel-argument image of a model (uniform across the grid).
struct KModel {
  int32_t n_gates, n_ch, v_method, has_syn;
  int32_t kind[kMaxGates];
  int32_t form[kMaxGates][2];
  KRate rate[kMaxGates][2];
  int32_t cexp[kMaxCh][kMaxGates];  // exponent of gate g in channel c (0 = absent)
  float gbar[kMaxCh], E[kMaxCh];
  float dt, v_th, C, kdt;           // kdt = -dt log2(e)
  float decay_e, decay_i, E_e, E_i; // synapse decay factors over one dt
};

// ---------------------------------------------------------------------------
// channel-set specs
//
// A spec tells the step code the *structure* of a channel set: number of
// gates and channels, each rate's form, each gate's kind and each channel's
// gate exponents.  GenericSpec reads them from the kernel arguments at run
// time (wave-uniform scalar branches).  FixedSpec carries them as template
// constants, so the compiler sees a straight-line program with the branches
// and unused paths removed.  Coefficients are run-time data in both cases.
// ---------------------------------------------------------------------------
template <int NG>
struct GenericSpec {
  static constexpr bool kFixed = false;
  static constexpr int kNG = NG;
  __device__ static int form(const KModel& M, int g, int r) { return M.form[g][r]; }
  __device__ static int kind(const KModel& M, int g) { return M.kind[g]; }
  __device__ static int nch(const KModel& M) { return M.n_ch; }
  __device__ static int cexp(const KModel& M, int c, int g) { return M.cexp[c][g]; }
};

// FORMS: 2 bits per rate at bit 2*(2g + r); KINDS: 1 bit per gate; Cc: 4 bits
// per gate exponent of channel c.
template <int NG, int NCH, uint32_t FORMS, uint32_t KINDS, uint32_t C0, uint32_t C1 = 0,
          uint32_t C2 = 0, uint32_t C3 = 0, uint32_t C4 = 0, uint32_t C5 = 0, uint32_t C6 = 0,
          uint32_t C7 = 0>
struct FixedSpec {
  static constexpr bool kFixed = true;
  static constexpr int kNG = NG;
  __host__ __device__ static constexpr int form(const KModel&, int g, int r) {
    return (int)((FORMS >> (2 * (2 * g + r))) & 3u);
  }
  __host__ __device__ static constexpr int kind(const KModel&, int g) { return (int)((KINDS >> g) & 1u); }
  __host__ __device__ static constexpr int nch(const KModel&) { return NCH; }
  __host__ __device__ static constexpr uint32_t cword(int c) {
    return c == 0 ? C0 : c == 1 ? C1 : c == 2 ? C2 : c == 3 ? C3 : c == 4 ? C4 : c == 5 ? C5 : c == 6 ? C6 : C7;
  }
  __host__ __device__ static constexpr int cexp(const KModel&, int c, int g) {
    return (int)((cword(c) >> (4 * g)) & 15u);
  }
  // does a run-time model have exactly this structure?
  static bool matches(const KModel& M) {
    if (M.n_gates != NG || M.n_ch != NCH) return false;
    for (int g = 0; g < NG; ++g) {
      if (M.kind[g] != kind(M, g)) return false;
      for (int r = 0; r < 2; ++r)
        if (M.form[g][r] != form(M, g, r)) return false;
    }
    for (int c = 0; c < NCH; ++c)
      for (int g = 0; g < kMaxGates; ++g)
        if (M.cexp[c][g] != (g < NG ? cexp(M, c, g) : 0)) return false;
    return true;
  }
};

// Hodgkin-Huxley (1952): m (linoid, exp), h (exp, sigmoid), n (linoid, exp);
// Na m^3 h, K n^4, leak.
using ClassicSpec = FixedSpec<3, 3,
    (2u << 0) | (0u << 2) | (0u << 4) | (1u << 6) | (2u << 8) | (0u << 10), 0u,
    0x13u, 0x400u, 0u>;
// Cortical set: m (linoid, linoid), h (exp, sigmoid), n (linoid, exp),
// p (sigmoid p_inf, bell 1/tau), q (linoid, exp); Na m^3 h, Kd n^4, M p,
// L-Ca q^2, leak.
using CorticalSpec = FixedSpec<5, 5,
    (2u << 0) | (2u << 2) | (0u << 4) | (1u << 6) | (2u << 8) | (0u << 10) | (1u << 12) |
        (3u << 14) | (2u << 16) | (0u << 18),
    1u << 3, 0x13u, 0x400u, 0x1000u, 0x20000u, 0u>;

// ---------------------------------------------------------------------------
// special-function unit
// ---------------------------------------------------------------------------
__device__ __forceinline__ float ex2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Rate value (and V-derivative when D) of one rate function.  `form` is
// uniform across the wavefront, so the switch is a scalar branch.
template <bool D>
__device__ __forceinline__ float rate_eval(int form, const KRate& k, float V, float* dr) {
  const float x = fmaf(V, k.s, k.o);
  float r;
  switch (form) {
    case FORM_EXP: {
      r = k.a * ex2(x);
      if (D) *dr = r * k.ik;
      break;
    }
    case FORM_SIGMOID: {
      const float q = rcp(1.0f + ex2(x));
      r = k.a * q;
      if (D) *dr = -r * k.ik * (1.0f - q);
      break;
    }
    case FORM_LINOID: {
      // g(u) = u / (1 - e^{-u}) has a removable singularity at u = 0.  Below
      // |u| = 1/4 its Bernoulli series (to u^4) is used: truncation < 1e-8,
      // while the direct quotient loses ~6e-8/|u| to cancellation.
      const float u = x * kLn2;
      const float E = ex2(-x);
      const float om = 1.0f - E;
      const float ro = rcp(om);
      const float u2 = u * u;
      const bool small = fabsf(u) < 0.25f;
      const float gs = fmaf(u, 0.5f, fmaf(u2, fmaf(u2, -1.0f / 720.0f, 1.0f / 12.0f), 1.0f));
      const float g = small ? gs : u * ro;
      r = k.a * g;
      if (D) {
        const float gps = fmaf(u, fmaf(u2, fmaf(u2, 1.0f / 5040.0f, -1.0f / 180.0f), 1.0f / 6.0f), 0.5f);
        const float gpd = (om - u * E) * ro * ro;
        *dr = k.a * k.ik * (small ? gps : gpd);
      }
      break;
    }
    default: {  // FORM_BELL
      const float ep = ex2(x), em = ex2(-x);
      r = k.a * fmaf(k.c, ep, em);
      if (D) *dr = k.a * k.ik * fmaf(k.c, ep, -em);
      break;
    }
  }
  return r;
}

// Derived constants of one rate from its (A, B, K, c) -- per-lane version
// for per-neuron coefficient tables.
__device__ __forceinline__ KRate derive_rate(int form, float A, float B, float K, float c) {
  KRate k;
  k.ik = 1.0f / K;
  k.s = kLog2e / K;
  k.o = -B * k.s;
  k.c = c;
  k.a = (form == FORM_LINOID) ? A * K : (form == FORM_BELL ? 1.0f / A : A);
  return k;
}

// Tabulated gate kinetics (the rate-function approximation lever of the
// method, Engineering: rates replaced by cheaper approximations).  For gate g
// and voltage node i (V_i = v_lo + i h), tab[g n + i] holds
//   { P(V_i), P(V_i+1) - P(V_i), Q(V_i), Q(V_i+1) - Q(V_i) }
// with P = p_inf and Q = 1 - e, the fraction of the way to p_inf that one
// exponential-Euler step covers.  Between nodes both are interpolated
// linearly in V; V outside [v_lo, v_lo + (n-1) h] is clamped to the range.
struct TabRates {
  const float4* tab;
  int n;
  float v_lo, inv_h;
};
template <class LR>
struct is_tab {
  static constexpr bool value = false;
};
template <>
struct is_tab<TabRates> {
  static constexpr bool value = true;
};

// A copy of x in a vector register that the compiler cannot re-derive from a
// scalar original: it then keeps the register for the whole loop instead of
// copying the scalar into a vector register at every use (a vector
// instruction reads at most one scalar operand).
__device__ __forceinline__ float pin_vgpr(float x) {
  float y;
  asm("v_mov_b32 %0, %1" : "=v"(y) : "v"(x));
  return y;
}

// Integer power with a wave-uniform exponent.
__device__ __forceinline__ float ipow(float p, int e) {
  switch (e) {
    case 0: return 1.0f;
    case 1: return p;
    case 2: return p * p;
    case 3: return p * p * p;
    case 4: { const float q = p * p; return q * q; }
    default: {
      float r = 1.0f;
      for (int j = 0; j < e; ++j) r *= p;
      return r;
    }
  }
}

// ---------------------------------------------------------------------------
// one neuron, one step (Jacobi: every right-hand side at the start state)
// ---------------------------------------------------------------------------
// Register arrays sized for NG gates (at least one slot so that leak-only
// models, NG = 0, still compile).
template <int NG>
constexpr int ng1 = NG > 0 ? NG : 1;

template <int NG>
struct LaneRates {
  KRate r[ng1<NG>][2];
};

template <class S>
__device__ __forceinline__ void load_rates(const KModel& M, const float* __restrict__ coef,
                                           int64_t pidx, int64_t N, LaneRates<S::kNG>& L) {
#pragma unroll
  for (int g = 0; g < S::kNG; ++g)
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      if (coef) {
        const float* cp = coef + (int64_t)(g * 8 + r * 4) * N + pidx;
        const int f = S::form(M, g, r);
        // the c coefficient only enters the bell form
        L.r[g][r] = derive_rate(f, cp[0], cp[N], cp[2 * N], f == FORM_BELL ? cp[3 * N] : 0.0f);
      } else {
        L.r[g][r] = M.rate[g][r];
      }
    }
}

// V is carried as an unevaluated sum vh + vl of two floats: the per-step
// change of V near rest is far below half an FP32 ulp of V (3.8e-6 mV at
// -65 mV), and rounding it into vh alone would stall slow subthreshold
// drift.  The increment is added with an exact two-sum.
__device__ __forceinline__ void add_to_v(float& vh, float& vl, float dv) {
  const float y = dv + vl;
  const float t = vh + y;
  const float bp = t - vh;
  const float ap = t - bp;
  vl = (vh - ap) + (y - bp);
  vh = t;
}

// Exponential-Euler gate step p' = p_inf + (p - p_inf) e (Methods, "Simplified
// discretization"), written as p + (p_inf - p)(1 - e): the fused multiply-add then
// accumulates into p itself, so the loop-carried register needs no copy.  The
// absolute error of e enters both forms the same way, times |p_inf - p|.
__device__ __forceinline__ float gate_update(float p, float pinf, float e) {
  return fmaf(pinf - p, 1.0f - e, p);
}

// e^{-z} - 1 for z >= 0 without cancellation at small z (series below 0.1,
// truncation < 2e-9 relative).
__device__ __forceinline__ float expm1_neg(float z) {
  // -z + z^2/2 - z^3/6 + z^4/24 - z^5/120
  const float s = z * fmaf(z, fmaf(z, fmaf(z, fmaf(z, -1.0f / 120.0f, 1.0f / 24.0f), -1.0f / 6.0f), 0.5f), -1.0f);
  return (z < 0.1f) ? s : ex2(-z * kLog2e) - 1.0f;
}

// 1 - e^{-z} for z >= 0 (the exponential-Euler gate increment q): the
// series z - z^2/2 + z^3/6 below 0.011 (truncation < 6e-8 relative), where
// 1 - e would cancel; beyond it 1 - e keeps its relative error below 1e-5.
__device__ __forceinline__ float one_minus_exp_neg(float z) {
  float q = z * fmaf(z, fmaf(z, 1.0f / 6.0f, -0.5f), 1.0f);
  if (z >= 0.011f) {
    // rare for slow gates: kept a branch (the empty asm stops the compiler
    // from evaluating it for every lane and selecting), so that its value
    // is never live beside the series
    asm volatile("");
    q = 1.0f - ex2(-z * kLog2e);
  }
  return q;
}

// Channel conductances g_X: the model's, the same for every neuron
// (ModelGbar), or one set per lane (LaneGbar: the compartments of a
// morphology, each with its own channel densities).
struct ModelGbar {
  __device__ __forceinline__ float operator()(const KModel& M, int c) const { return M.gbar[c]; }
};
struct LaneGbar {
  float g[kMaxCh];
  __device__ __forceinline__ float operator()(const KModel&, int c) const { return g[c]; }
};

// One compartment of a morphology, shared by every neuron of a population
// (Methods, Eq. (1): the spatial term, discretized by the second-order
// explicit difference).  par / ch: compartment indices (within the neuron)
// of the parent and of up to kMaxChildren children, the compartment's own
// index where there is none (the term then vanishes).  gup / gdn: the
// coupling coefficients g_edge / area of this compartment towards each of
// them (mS/cm^2).  gbar: the compartment's channel conductances.
constexpr int kMaxChildren = 4;
struct CableComp {
  int32_t par, ch[kMaxChildren];
  float gup, gdn[kMaxChildren];
  float gbar[kMaxCh];
};

// Advance the gates and V by one step (Jacobi: all right-hand sides at the
// start-of-step state).  p is updated in place; (vh, vl) likewise.
// I: external current; ge, gi: synaptic conductances held over the step.
// SYN = false: the caller knows the population has no synapses (ge = gi = 0);
// the synaptic terms are left out, which gives bit-identical results.  LR:
// LaneRates (rate functions) or TabRates (tabulated gate kinetics).  GB:
// where the channel conductances come from (ModelGbar or LaneGbar).
template <class S, bool SYN = true, class LR = LaneRates<S::kNG>, class GB = ModelGbar>
__device__ __forceinline__ void neuron_step(const KModel& M, const LR& L, float dtC,
                                            float& vh, float& vl, float (&p)[ng1<S::kNG>], float I,
                                            float ge, float gi, const GB& G = GB()) {
  constexpr int NG = S::kNG;
  const float V = vh;
  // channel terms at the start-of-step gates: total conductance gsum and
  // sum of g_X E_X, so that I_ion + I_syn = gsum V - esum
  float gsum = 0.0f, esum = 0.0f;
  if constexpr (SYN) {
    gsum = ge + gi;
    esum = fmaf(ge, M.E_e, gi * M.E_i);
  }
#pragma unroll
  for (int c = 0; c < kMaxCh; ++c) {
    if (c >= S::nch(M)) break;
    float eta = G(M, c);
#pragma unroll
    for (int g = 0; g < NG; ++g) {
      const int e = S::cexp(M, c, g);
      if (e) eta *= ipow(p[g], e);
    }
    gsum += eta;
    esum = fmaf(eta, M.E[c], esum);
  }
  // gates by exponential Euler at V_t
  if constexpr (is_tab<LR>::value) {
    // one voltage index for all gates, then per gate one 16-byte table read
    const float u = fminf(fmaxf((V - L.v_lo) * L.inv_h, 0.0f), (float)(L.n - 1));
    const int ix = min((int)u, L.n - 2);
    const float t = u - (float)ix;
#pragma unroll
    for (int g = 0; g < NG; ++g) {
      const float4 c = L.tab[g * L.n + ix];
      const float P = fmaf(c.y, t, c.x), Q = fmaf(c.w, t, c.z);
      p[g] = fmaf(P - p[g], Q, p[g]);
    }
  } else {
#pragma unroll
    for (int g = 0; g < NG; ++g) {
      const float r0 = rate_eval<false>(S::form(M, g, 0), L.r[g][0], V, nullptr);
      const float r1 = rate_eval<false>(S::form(M, g, 1), L.r[g][1], V, nullptr);
      if (S::kind(M, g) == KIND_AB) {
        const float s = r0 + r1;
        p[g] = gate_update(p[g], r0 * rcp(s), ex2(s * M.kdt));
      } else {
        // (p_inf, 1/tau) gates carry the slow kinetics (tau up to seconds):
        // there e^{-dt/tau} lies within a few ulps of 1, and 1 - e formed from
        // it would lose most of its digits, so q = 1 - e comes from the series
        p[g] = fmaf(r0 - p[g], one_minus_exp_neg(r1 * M.dt), p[g]);
      }
    }
  }
  // membrane
  float dv;
  if (M.v_method == VFE) {
    const float iion = fmaf(gsum, vl, fmaf(gsum, V, -esum));
    dv = dtC * (I - iion);
  } else {
    // V' - V = (V - V_inf) (e^{-dt gsum / C} - 1)
    const float vinf = (I + esum) * rcp(gsum);
    dv = ((V - vinf) + vl) * expm1_neg(gsum * dtC);
  }
  add_to_v(vh, vl, dv);
}

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11) and Box-Muller
// ---------------------------------------------------------------------------
struct U4 {
  uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox10(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
    U4 n;
    n.x = (uint32_t)(p1 >> 32) ^ c.y ^ k0;
    n.y = (uint32_t)p1;
    n.z = (uint32_t)(p0 >> 32) ^ c.w ^ k1;
    n.w = (uint32_t)p0;
    c = n;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

// Four standard normals of the noise block (seed, id, blk): Box-Muller on
// word pairs, u = (w + 1/2) 2^-32.
__device__ __forceinline__ void normals4(uint64_t seed, uint32_t id, uint64_t blk, float (&z)[4]) {
  U4 c = {(uint32_t)blk, (uint32_t)(blk >> 32), id, 0u};
  const U4 w = philox10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
  const float s = 2.3283064365386963e-10f;  // 2^-32
  const float h = 1.1641532182693481e-10f;  // 2^-33
  const float u0 = fmaf((float)w.x, s, h), u1 = fmaf((float)w.y, s, h);
  const float u2 = fmaf((float)w.z, s, h), u3 = fmaf((float)w.w, s, h);
  // -2 ln u = -2 ln2 log2 u
  const float ra = __builtin_amdgcn_sqrtf(-2.0f * kLn2 * __builtin_amdgcn_logf(u0));
  const float rb = __builtin_amdgcn_sqrtf(-2.0f * kLn2 * __builtin_amdgcn_logf(u2));
  // v_cos_f32 / v_sin_f32 take revolutions: cos(2 pi u)
  z[0] = ra * __builtin_amdgcn_cosf(u1);
  z[1] = ra * __builtin_amdgcn_sinf(u1);
  z[2] = rb * __builtin_amdgcn_cosf(u3);
  z[3] = rb * __builtin_amdgcn_sinf(u3);
}

// Background input (Methods, cortical network), drawn directly: N ~
// Poisson(lam) events of Gaussian amplitude (mu, sigma), N mu + sqrt(N) sigma
// z.  N is an integer decided by floating point, so its inverse-transform
// search uses only correctly rounded binary32 operations, each rounded on
// its own (contraction off), from p0 = e^-lam rounded once on the host;
// u = (2 floor(w0 / 2^9) + 1) 2^-24 is exact in binary32.
__device__ __forceinline__ int background_count(uint32_t w0, float lam, float p0, int kmax) {
#pragma clang fp contract(off)
  const float u = (float)(2u * (w0 >> 9) + 1u) * 0x1p-24f;
  int k = 0;
  float p = p0, F = p0;
  while (u > F && k < kmax) {
    ++k;
    p = p * (lam / (float)k);
    F = F + p;
  }
  return k;
}

__device__ __forceinline__ float background_current(uint64_t seed, uint32_t id, uint64_t t,
                                                    float lam, float p0, int kmax, float mu,
                                                    float sigma) {
  U4 c = {(uint32_t)t, (uint32_t)(t >> 32), id, 2u};
  const U4 w = philox10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
  const float fk = (float)background_count(w.x, lam, p0, kmax);
  const float s = 2.3283064365386963e-10f;  // 2^-32
  const float h = 1.1641532182693481e-10f;  // 2^-33
  const float ua = fmaf((float)w.z, s, h), ub = fmaf((float)w.w, s, h);
  const float z = __builtin_amdgcn_sqrtf(-2.0f * kLn2 * __builtin_amdgcn_logf(ua)) *
                  __builtin_amdgcn_cosf(ub);
  return fmaf(fk, mu, __builtin_amdgcn_sqrtf(fk) * sigma * z);
}

// Sinusoidal input (Results, HH encryption): R = round(f K) revolutions / 2^32
// per step (f K in binary32; clamped below 2^32), the phase of step t the
// wrapped product R t, exact; v_sin_f32 takes the phase in revolutions.
__device__ __forceinline__ uint32_t sine_rate(float f, float K) {
  return (uint32_t)rintf(fminf(fmaxf(f * K, 0.0f), 4294967040.0f));
}
// the input at phase ph (revolutions / 2^32): a caller that starts at
// ph = R t0 and adds R per step (wrapping) has ph = R t mod 2^32 exactly
__device__ __forceinline__ float sine_input(float amp, uint32_t ph) {
  return amp * __builtin_amdgcn_sinf((float)ph * 0x1p-32f);
}

__device__ __forceinline__ uint32_t event_word(uint64_t seed, uint32_t id, uint64_t t) {
  U4 c = {(uint32_t)t, (uint32_t)(t >> 32), id, 1u};
  return philox10(c, (uint32_t)seed, (uint32_t)(seed >> 32)).x;
}

}  // namespace hhk
