/*
 * hh_oracle.c -- FP64 reference integrator for Hodgkin-Huxley populations.
 *
 * TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test suite, the smoke entry
 * and the CPU-baseline leg of the benchmark may load it.  It shares no code
 * with the HIP library.  Plain single-threaded double precision.
 *
 * The model (Methods, "Membrane potential and ion-channel definitions",
 * Eq. (1)), point-neuron form (cable term dropped):
 *     C dV/dt = I - sum_X gbar_X eta_X(p) (V - E_X) - I_syn
 *     dp/dt   = alpha_p(V) (1 - p) - beta_p(V) p
 * eta_X is a product of integer powers of gate variables.  The sign of the
 * ionic term is the physical one; Eq. (2) folds it into f(V, t).
 *
 * Discretization ("Simplified discretization"): exponential Euler for the
 * gate equations, explicit Euler for V (Eq. (2)) or, optionally, exponential
 * Euler in V.  Every right-hand side of one step uses the values at the start
 * of that step (the step is a pure map x_{t+1} = F(x_t, I_t)).
 */
#include "hh_oracle.h"

#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------------------
 * Philox4x32-10, as defined by Salmon et al., "Parallel random numbers: as
 * easy as 1, 2, 3" (SC'11): ten rounds of two 32x32->64 multiplies with the
 * published multipliers, the key bumped by the published Weyl constants
 * between rounds.
 * ------------------------------------------------------------------------- */
void ora_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t y0 = hi1 ^ x1 ^ k0;
    uint32_t y1 = lo1;
    uint32_t y2 = hi0 ^ x3 ^ k1;
    uint32_t y3 = lo0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Uniform on (0, 1) from a 32-bit word: (w + 1/2) / 2^32. */
static double unit_open(uint32_t w) { return ((double)w + 0.5) * (1.0 / 4294967296.0); }

/* Box-Muller: two uniforms give two independent standard normals,
 * sqrt(-2 ln u0) cos(2 pi u1) and sqrt(-2 ln u0) sin(2 pi u1). */
double ora_noise(uint64_t seed, uint32_t id, int64_t t) {
  uint64_t blk = (uint64_t)t >> 2;
  uint32_t ctr[4] = {(uint32_t)blk, (uint32_t)(blk >> 32), id, 0u};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t w[4];
  ora_philox4x32_10(ctr, key, w);
  int comp = (int)(t & 3);
  const double two_pi = 6.283185307179586476925286766559;
  double ua = unit_open(w[(comp >> 1) * 2]);
  double ub = unit_open(w[(comp >> 1) * 2 + 1]);
  double rad = sqrt(-2.0 * log(ua));
  return (comp & 1) ? rad * sin(two_pi * ub) : rad * cos(two_pi * ub);
}

/* Background input of the cortex model (Methods, cortical network): the
 * summed drive of many background synapses over one step, drawn directly
 * from its distribution instead of synapse by synapse.  Read as a compound
 * Poisson sum: N ~ Poisson(lam) events in the step, each of independent
 * Gaussian amplitude (mu, sigma), so the sum is N mu + sqrt(N) sigma z.
 *
 * The random words are block (t, stream 2) of Philox4x32-10 for the element.
 * Word 0 gives u = (2 floor(w0 / 2^9) + 1) 2^-24, which binary32 holds
 * exactly, and N is the smallest k with u <= F(k), by sequential search.
 * N is an integer that floating point decides, so the search runs in
 * binary32 like the device kernel: every product, quotient and sum is
 * rounded to binary32 on its own, and p_0 = e^-lam is rounded once from
 * binary64.  The search stops at k_max = floor(lam + 12 sqrt(lam)) + 12.
 * Words 2 and 3 give z by Box-Muller (cosine branch). */
int32_t ora_background_count(uint32_t w0, double lam) {
  const float u = (float)(2u * (w0 >> 9) + 1u) * 0x1p-24f;
  const float lf = (float)lam;
  const float p0 = (float)exp(-lam);
  const int32_t kmax = (int32_t)floor(lam + 12.0 * sqrt(lam)) + 12;
  int32_t k = 0;
  float p = p0, F = p0;
  /* binary32 arithmetic; the oracle is built without contraction, so each
   * operation is rounded on its own */
  while (u > F && k < kmax) {
    k += 1;
    p = p * (lf / (float)k);
    F = F + p;
  }
  return k;
}

double ora_background(uint64_t seed, uint32_t id, int64_t t, double lam, double mu, double sigma,
                      int32_t* count) {
  uint32_t ctr[4] = {(uint32_t)(uint64_t)t, (uint32_t)((uint64_t)t >> 32), id, 2u};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t w[4];
  ora_philox4x32_10(ctr, key, w);
  const int32_t N = ora_background_count(w[0], lam);
  const double two_pi = 6.283185307179586476925286766559;
  const double z = sqrt(-2.0 * log(unit_open(w[2]))) * cos(two_pi * unit_open(w[3]));
  if (count) *count = N;
  return (double)N * mu + sqrt((double)N) * sigma * z;
}

/* Sinusoidal input (Results, HH encryption).  The phase advances by R / 2^32
 * revolutions per step with R the binary32 product f * K rounded to an
 * integer, so that R t wraps exactly in 32-bit arithmetic. */
uint32_t ora_sine_rate(double f, double dt) {
  const float K = (float)(dt * 4294967296.0 / 1000.0);
  const float x = (float)f * K;
  return (uint32_t)lrintf(x);
}

double ora_sine(double amp, uint32_t R, int64_t t) {
  const uint32_t ph = R * (uint32_t)(uint64_t)t; /* mod 2^32 */
  return amp * sin(6.283185307179586476925286766559 * ((double)ph / 4294967296.0));
}

uint32_t ora_event_word(uint64_t seed, uint32_t id, int64_t t) {
  uint32_t ctr[4] = {(uint32_t)(uint64_t)t, (uint32_t)((uint64_t)t >> 32), id, 1u};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t w[4];
  ora_philox4x32_10(ctr, key, w);
  return w[0];
}

/* ---------------------------------------------------------------------------
 * Rate functions (the alpha_p(V), beta_p(V) of Eq. (1)) and their
 * derivatives in V.
 * ------------------------------------------------------------------------- */
double ora_rate(int32_t form, const double k[4], double V, double* dV) {
  const double A = k[0], B = k[1], K = k[2], c = k[3];
  const double u = (V - B) / K;
  double r = 0.0, d = 0.0;
  switch (form) {
    case ORA_EXP:
      r = A * exp(u);
      d = r / K;
      break;
    case ORA_SIGMOID: {
      double e = exp(u);
      r = A / (1.0 + e);
      d = -A * e / ((1.0 + e) * (1.0 + e)) / K;
      break;
    }
    case ORA_LINOID: {
      /* A (V - B) / (1 - e^{-u}) = A K g(u), g(u) = u / (1 - e^{-u}).
       * At small |u| the Bernoulli series g = 1 + u/2 + u^2/12 - u^4/720
       * replaces the 0/0 form; its truncation error there is below 1e-19. */
      double g, gp;
      if (fabs(u) < 1e-3) {
        g = 1.0 + u / 2.0 + u * u / 12.0 - u * u * u * u / 720.0;
        gp = 0.5 + u / 6.0 - u * u * u / 180.0;
      } else {
        double om = -expm1(-u); /* 1 - e^{-u} */
        double E = exp(-u);
        g = u / om;
        gp = (om - u * E) / (om * om);
      }
      r = A * K * g;
      d = A * gp;
      break;
    }
    case ORA_BELL: {
      double ep = exp(u), em = exp(-u);
      r = (c * ep + em) / A;
      d = (c * ep - em) / (A * K);
      break;
    }
    default:
      r = NAN;
      d = NAN;
  }
  if (dV) *dV = d;
  return r;
}

int32_t ora_n_state(const ora_model* m) { return 1 + m->n_gates + (m->has_syn ? 2 : 0); }

static void coefs_of(const ora_model* m, const double* coef, int64_t n, int64_t i, int32_t g,
                     int32_t r, double k[4]) {
  for (int j = 0; j < 4; ++j)
    k[j] = coef ? coef[(int64_t)(g * 8 + r * 4 + j) * n + i] : m->rate_coef[g][r][j];
}

/* Gate g at V: steady state p_inf, decay factor e over one dt, and their V
 * derivatives.  Exponential Euler ("Simplified discretization") holds V fixed
 * over the step, so p' = p_inf + (p - p_inf) e is the exact solution of the
 * gate equation for that step. */
static void gate_terms(const ora_model* m, const double* coef, int64_t n, int64_t i, int32_t g,
                       double V, double* pinf, double* e, double* dpinf, double* de) {
  double k0[4], k1[4], d0, d1;
  coefs_of(m, coef, n, i, g, 0, k0);
  coefs_of(m, coef, n, i, g, 1, k1);
  double r0 = ora_rate(m->rate_form[g][0], k0, V, &d0);
  double r1 = ora_rate(m->rate_form[g][1], k1, V, &d1);
  const double dt = m->dt;
  if (m->gate_kind[g] == ORA_AB) {
    double s = r0 + r1;
    *pinf = r0 / s;
    *e = exp(-dt * s);
    *dpinf = (d0 * r1 - r0 * d1) / (s * s);
    *de = -dt * (d0 + d1) * (*e);
  } else {
    *pinf = r0;
    *e = exp(-dt * r1);
    *dpinf = d0;
    *de = -dt * d1 * (*e);
  }
}

double ora_gate_inf(const ora_model* m, const double* coef, int64_t n, int64_t i, int32_t g,
                    double V) {
  double pinf, e, dp, de;
  gate_terms(m, coef, n, i, g, V, &pinf, &e, &dp, &de);
  return pinf;
}

/* Exact exponential-Euler terms of gate g at V: P = p_inf, Q = 1 - e. */
static void exact_pq(const ora_model* m, const double* coef, int64_t n, int64_t i, int32_t g,
                     double V, double* P, double* Q) {
  double pinf, e, dp, de;
  gate_terms(m, coef, n, i, g, V, &pinf, &e, &dp, &de);
  *P = pinf;
  *Q = 1.0 - e;
}

/* Tabulated kinetics: the exact P and Q at the nodes v_k = tab_vlo + k tab_h,
 * joined by straight lines.  u = (V - tab_vlo) / tab_h locates V; it is
 * clamped to [0, tab_n - 1], so V beyond either end takes the end node's
 * values; the segment is k = floor(u) (the last segment at the top node) and
 * t = u - k the position inside it. */
void ora_gate_pq(const ora_model* m, const double* coef, int64_t n, int64_t i, int32_t g,
                 double V, double* P, double* Q) {
  if (m->tab_n < 2) {
    exact_pq(m, coef, n, i, g, V, P, Q);
    return;
  }
  double u = (V - m->tab_vlo) / m->tab_h;
  if (u < 0.0) u = 0.0;
  if (u > (double)(m->tab_n - 1)) u = (double)(m->tab_n - 1);
  int64_t k = (int64_t)floor(u);
  if (k > m->tab_n - 2) k = m->tab_n - 2;
  const double t = u - (double)k;
  double Pa, Qa, Pb, Qb;
  exact_pq(m, coef, n, i, g, m->tab_vlo + (double)k * m->tab_h, &Pa, &Qa);
  exact_pq(m, coef, n, i, g, m->tab_vlo + (double)(k + 1) * m->tab_h, &Pb, &Qb);
  *P = Pa + t * (Pb - Pa);
  *Q = Qa + t * (Qb - Qa);
}

void ora_init_state(const ora_model* m, const double* coef, int64_t n, const double* v0,
                    double* state) {
  for (int64_t i = 0; i < n; ++i) {
    state[i] = v0[i];
    for (int g = 0; g < m->n_gates; ++g)
      state[(int64_t)(1 + g) * n + i] = ora_gate_inf(m, coef, n, i, g, v0[i]);
    if (m->has_syn) {
      state[(int64_t)(1 + m->n_gates) * n + i] = 0.0;
      state[(int64_t)(2 + m->n_gates) * n + i] = 0.0;
    }
  }
}

static int model_ok(const ora_model* m) {
  if (m->n_gates < 0 || m->n_gates > ORA_MAX_GATES) return 0;
  if (m->n_channels < 0 || m->n_channels > ORA_MAX_CH) return 0;
  for (int c = 0; c < m->n_channels; ++c) {
    if (m->ch_n[c] < 0 || m->ch_n[c] > 4) return 0;
    for (int k = 0; k < m->ch_n[c]; ++k)
      if (m->ch_gate[c][k] < 0 || m->ch_gate[c][k] >= m->n_gates || m->ch_expo[c][k] < 0) return 0;
  }
  if (m->tab_n < 0 || m->tab_n == 1 || (m->tab_n >= 2 && !(m->tab_h > 0.0))) return 0;
  return m->dt > 0.0;
}

/* Open fraction eta_X(p) = prod_k p_{g_k}^{a_k} of channel c, and its partial
 * derivatives d eta / d p_g (accumulated into deta[g] if non-null). */
static double channel_eta(const ora_model* m, int c, const double* p, double* deta) {
  double eta = 1.0;
  for (int k = 0; k < m->ch_n[c]; ++k) eta *= pow(p[m->ch_gate[c][k]], (double)m->ch_expo[c][k]);
  if (deta) {
    for (int g = 0; g < m->n_gates; ++g) deta[g] = 0.0;
    for (int k = 0; k < m->ch_n[c]; ++k) {
      int a = m->ch_expo[c][k];
      if (a == 0) continue;
      double term = a * pow(p[m->ch_gate[c][k]], (double)(a - 1));
      for (int k2 = 0; k2 < m->ch_n[c]; ++k2)
        if (k2 != k) term *= pow(p[m->ch_gate[c][k2]], (double)m->ch_expo[c][k2]);
      deta[m->ch_gate[c][k]] += term;
    }
  }
  return eta;
}

/* One step of one neuron: x = (V, p[0..G-1]) at time t, synaptic
 * conductances ge, gi held over the step, external current I.  Writes the
 * state at t+1 into Vn, pn. */
static void neuron_step(const ora_model* m, const double* coef, int64_t n, int64_t i, double C,
                        double V, const double* p, double ge, double gi, double I, double* Vn,
                        double* pn) {
  for (int g = 0; g < m->n_gates; ++g) {
    if (m->tab_n >= 2) {
      double P, Q;
      ora_gate_pq(m, coef, n, i, g, V, &P, &Q);
      pn[g] = p[g] + (P - p[g]) * Q;
    } else {
      double pinf, e, dp, de;
      gate_terms(m, coef, n, i, g, V, &pinf, &e, &dp, &de);
      pn[g] = pinf + (p[g] - pinf) * e;
    }
  }
  if (m->v_method == ORA_FE) {
    double i_ion = 0.0;
    for (int c = 0; c < m->n_channels; ++c)
      i_ion += m->ch_gbar[c] * channel_eta(m, c, p, NULL) * (V - m->ch_E[c]);
    double i_syn = ge * (V - m->E_e) + gi * (V - m->E_i);
    *Vn = V + (m->dt / C) * (I - i_ion - i_syn);
  } else {
    double gtot = ge + gi, num = I + ge * m->E_e + gi * m->E_i;
    for (int c = 0; c < m->n_channels; ++c) {
      double gx = m->ch_gbar[c] * channel_eta(m, c, p, NULL);
      gtot += gx;
      num += gx * m->ch_E[c];
    }
    double vinf = num / gtot;
    *Vn = vinf + (V - vinf) * exp(-m->dt * gtot / C);
  }
}

static int32_t run_impl(const ora_model* m, int64_t n, const double* coef, const double* cm,
                        const uint32_t* ids, double* state, int64_t t0, int32_t T,
                        int32_t in_mode, const double* i_const, double mu, double sigma,
                        uint64_t seed, double lam, const double* freq, const double* i_dense,
                        uint8_t* spk, double* vrec, double* level);

/* Threads the parallel loops use: 1 in the serial build. */
int32_t ora_threads(void) {
#ifdef _OPENMP
  return (int32_t)omp_get_max_threads();
#else
  return 1;
#endif
}

int32_t ora_run(const ora_model* m, int64_t n, const double* coef, const double* cm,
                const uint32_t* ids, double* state, int64_t t0, int32_t T, int32_t in_mode,
                const double* i_const, double mu, double sigma, uint64_t seed, double lam,
                const double* i_dense, uint8_t* spk, double* vrec, double* level) {
  if (in_mode == ORA_IN_SINE) return -1; /* needs the frequencies: ora_run_sine */
  return run_impl(m, n, coef, cm, ids, state, t0, T, in_mode, i_const, mu, sigma, seed, lam, NULL,
                  i_dense, spk, vrec, level);
}

int32_t ora_run_sine(const ora_model* m, int64_t n, const double* coef, const double* cm,
                     double* state, int64_t t0, int32_t T, const double* amp, const double* freq,
                     uint8_t* spk, double* vrec, double* level) {
  return run_impl(m, n, coef, cm, NULL, state, t0, T, ORA_IN_SINE, amp, 0.0, 0.0, 0, 0.0, freq,
                  NULL, spk, vrec, level);
}

static int32_t run_impl(const ora_model* m, int64_t n, const double* coef, const double* cm,
                        const uint32_t* ids, double* state, int64_t t0, int32_t T,
                        int32_t in_mode, const double* i_const, double mu, double sigma,
                        uint64_t seed, double lam, const double* freq, const double* i_dense,
                        uint8_t* spk, double* vrec, double* level) {
  if (!model_ok(m) || n < 0 || T < 0) return -1;
  const int G = m->n_gates;
  /* neurons are independent: the OpenMP build of this same source (the
   * all-core timing leg) splits them over threads; every neuron's
   * arithmetic is unchanged */
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
  for (int64_t i = 0; i < n; ++i) {
    double V = state[i], p[ORA_MAX_GATES], pn[ORA_MAX_GATES], ge = 0.0, gi = 0.0;
    for (int g = 0; g < G; ++g) p[g] = state[(int64_t)(1 + g) * n + i];
    if (m->has_syn) {
      ge = state[(int64_t)(1 + G) * n + i];
      gi = state[(int64_t)(2 + G) * n + i];
    }
    const double C = cm ? cm[i] : m->C;
    const uint32_t id = ids ? ids[i] : (uint32_t)i;
    const double de = m->has_syn ? exp(-m->dt / m->tau_e) : 1.0;
    const double di = m->has_syn ? exp(-m->dt / m->tau_i) : 1.0;
    for (int32_t k = 0; k < T; ++k) {
      const int64_t t = t0 + k;
      double I = 0.0;
      if (in_mode == ORA_IN_CONST) I = i_const[i];
      else if (in_mode == ORA_IN_NOISE) I = mu + sigma * ora_noise(seed, id, t);
      else if (in_mode == ORA_IN_DENSE) I = i_dense[(int64_t)k * n + i];
      else if (in_mode == ORA_IN_BACKGROUND) I = ora_background(seed, id, t, lam, mu, sigma, NULL);
      else if (in_mode == ORA_IN_SINE) I = ora_sine(i_const[i], ora_sine_rate(freq[i], m->dt), t);
      double Vn;
      neuron_step(m, coef, n, i, C, V, p, ge, gi, I, &Vn, pn);
      if (spk) spk[(int64_t)k * n + i] = (uint8_t)(V < m->v_th && Vn >= m->v_th);
      if (vrec) vrec[(int64_t)k * n + i] = Vn;
      if (level && Vn >= m->v_th) level[i] += 1.0;
      V = Vn;
      for (int g = 0; g < G; ++g) p[g] = pn[g];
      ge *= de;
      gi *= di;
    }
    state[i] = V;
    for (int g = 0; g < G; ++g) state[(int64_t)(1 + g) * n + i] = p[g];
    if (m->has_syn) {
      state[(int64_t)(1 + G) * n + i] = ge;
      state[(int64_t)(2 + G) * n + i] = gi;
    }
  }
  return 0;
}

/* Multi-compartment neurons (Methods, Eq. (1) with the spatial term
 * (1/r_l) d2V/dx2; "Simplified discretization": a second-order explicit
 * difference in space).  Compartment c of neuron j is element j*K + c.  The
 * edge between c and parent[c] has conductance g_axial[c] per unit reference
 * area; the current it carries into compartment x (one of its two ends) per
 * unit of x's area is g_axial[c] / area[x] (V_other - V_x), so the charge
 * sum_x area[x] C V_x is conserved by the coupling.  All potentials are
 * those at the start of the step (explicit), and each compartment then takes
 * the point-neuron step with I + I_axial as its input.  gbar [K][n_channels]
 * (nullable) replaces the channel conductances per compartment; coef
 * (nullable) holds per-element rate coefficients and ids (nullable) the
 * noise generator's element ids, as in ora_run.  The steps
 * run in time order, all compartments within each step. */
int32_t ora_cable_run(const ora_model* m, int64_t n, int32_t K, const int32_t* parent,
                      const double* g_axial, const double* area, const double* gbar,
                      const double* coef, const double* cm, const uint32_t* ids, double* state,
                      int64_t t0, int32_t T, int32_t in_mode, const double* i_const, double mu,
                      double sigma, uint64_t seed, double lam, const double* i_dense, uint8_t* spk,
                      double* vrec) {
  if (!model_ok(m) || K < 1 || n < 0 || T < 0 || n % K != 0) return -1;
  for (int32_t c = 0; c < K; ++c)
    if (parent[c] < -1 || parent[c] >= c) return -1;
  const int G = m->n_gates;
  double* Vt = (double*)malloc(sizeof(double) * (size_t)(n ? n : 1));
  double* iax = (double*)malloc(sizeof(double) * (size_t)(n ? n : 1));
  ora_model* mc = (ora_model*)malloc(sizeof(ora_model) * (size_t)K);
  if (!Vt || !iax || !mc) {
    free(Vt);
    free(iax);
    free(mc);
    return -2;
  }
  for (int32_t c = 0; c < K; ++c) {
    mc[c] = *m;
    if (gbar)
      for (int x = 0; x < m->n_channels; ++x) mc[c].ch_gbar[x] = gbar[(int64_t)c * m->n_channels + x];
  }
  const double de = m->has_syn ? exp(-m->dt / m->tau_e) : 1.0;
  const double di = m->has_syn ? exp(-m->dt / m->tau_i) : 1.0;
  for (int32_t k = 0; k < T; ++k) {
    const int64_t t = t0 + k;
    for (int64_t i = 0; i < n; ++i) {
      Vt[i] = state[i];
      iax[i] = 0.0;
    }
    /* every edge adds to both of its ends */
    for (int64_t j = 0; j < n / K; ++j)
      for (int32_t c = 0; c < K; ++c) {
        const int32_t p = parent[c];
        if (p < 0) continue;
        const int64_t ic = j * K + c, ip = j * K + p;
        const double ac = area ? area[c] : 1.0, ap = area ? area[p] : 1.0;
        iax[ic] += g_axial[c] / ac * (Vt[ip] - Vt[ic]);
        iax[ip] += g_axial[c] / ap * (Vt[ic] - Vt[ip]);
      }
    for (int64_t i = 0; i < n; ++i) {
      const ora_model* mi = &mc[i % K];
      double V = state[i], p[ORA_MAX_GATES], pn[ORA_MAX_GATES], ge = 0.0, gi = 0.0;
      for (int g = 0; g < G; ++g) p[g] = state[(int64_t)(1 + g) * n + i];
      if (m->has_syn) {
        ge = state[(int64_t)(1 + G) * n + i];
        gi = state[(int64_t)(2 + G) * n + i];
      }
      double I = 0.0;
      if (in_mode == ORA_IN_CONST) I = i_const[i];
      else if (in_mode == ORA_IN_NOISE) I = mu + sigma * ora_noise(seed, ids ? ids[i] : (uint32_t)i, t);
      else if (in_mode == ORA_IN_DENSE) I = i_dense[(int64_t)k * n + i];
      else if (in_mode == ORA_IN_BACKGROUND)
        I = ora_background(seed, ids ? ids[i] : (uint32_t)i, t, lam, mu, sigma, NULL);
      double Vn;
      neuron_step(mi, coef, n, i, cm ? cm[i] : m->C, V, p, ge, gi, I + iax[i], &Vn, pn);
      if (spk) spk[(int64_t)k * n + i] = (uint8_t)(V < m->v_th && Vn >= m->v_th);
      if (vrec) vrec[(int64_t)k * n + i] = Vn;
      state[i] = Vn;
      for (int g = 0; g < G; ++g) state[(int64_t)(1 + g) * n + i] = pn[g];
      if (m->has_syn) {
        state[(int64_t)(1 + G) * n + i] = ge * de;
        state[(int64_t)(2 + G) * n + i] = gi * di;
      }
    }
  }
  free(Vt);
  free(iax);
  free(mc);
  return 0;
}

void ora_syn_deliver(int64_t n, const int64_t* row_ptr, const int32_t* col, const double* w,
                     double w_scale, const uint8_t* s, double* ge, double* gi) {
  for (int64_t j = 0; j < n; ++j) {
    if (!s[j]) continue;
    for (int64_t q = row_ptr[j]; q < row_ptr[j + 1]; ++q) {
      double x = w[q];
      if (x > 0.0) ge[col[q]] += w_scale * x;
      else if (x < 0.0) gi[col[q]] += w_scale * (-x);
    }
  }
}

/* Recurrent network.  Each step: every neuron advances with its conductances
 * held at time t (input: none, constant, or the background input); a neuron
 * spikes on an upward crossing of v_th; then
 *   g_e(t+1) = g_e(t) e^{-dt/tau_e} + scale * sum of w>0 over the synapses
 *              whose source spiked at t + 1 - d (d the synapse's delay in
 *              steps, 1 without a delay table) + w_ext * (external event at t+1),
 *   g_i(t+1) likewise with |w| of w<0 and no external term.
 * Arrivals due after the last step are dropped.  External events: driven
 * neurons (ext_mask) get a Bernoulli event when the stream-1 Philox word for
 * (id, t+1) is below ext_thresh. */
int32_t ora_net_run(const ora_model* m, int64_t n, double* state, const int64_t* row_ptr,
                    const int32_t* col, const double* w, double w_scale, const uint8_t* delay,
                    int32_t max_delay, const uint8_t* ext_mask, uint32_t ext_thresh, double w_ext,
                    uint64_t seed, int32_t in_mode, const double* i_const, double mu, double sigma,
                    uint64_t in_seed, double lam, int64_t t0, int32_t T, uint8_t* spk) {
  if (!model_ok(m) || !m->has_syn || n < 0 || T < 0) return -1;
  if (!delay) max_delay = 1;
  if (max_delay < 1) return -1;
  const int G = m->n_gates;
  const int R = max_delay + 1; /* arrival slots: times t+1 .. t+max_delay, and t */
  double* V = state;
  double* ge = state + (int64_t)(1 + G) * n;
  double* gi = state + (int64_t)(2 + G) * n;
  uint8_t* s = (uint8_t*)calloc((size_t)n + 1, 1);
  double* pend_e = (double*)calloc((size_t)R * (size_t)n + 1, sizeof(double));
  double* pend_i = (double*)calloc((size_t)R * (size_t)n + 1, sizeof(double));
  if (!s || !pend_e || !pend_i) {
    free(s); free(pend_e); free(pend_i);
    return -2;
  }
  const double de = exp(-m->dt / m->tau_e), di = exp(-m->dt / m->tau_i);
  for (int32_t k = 0; k < T; ++k) {
    const int64_t t = t0 + k;
    /* the neuron updates of a step are independent (the OpenMP build splits
     * them over threads; the synaptic sums below stay sequential) */
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
    for (int64_t i = 0; i < n; ++i) {
      double p[ORA_MAX_GATES], pn[ORA_MAX_GATES], Vn;
      for (int g = 0; g < G; ++g) p[g] = state[(int64_t)(1 + g) * n + i];
      double I = 0.0;
      if (in_mode == ORA_IN_CONST) I = i_const[i];
      else if (in_mode == ORA_IN_BACKGROUND) I = ora_background(in_seed, (uint32_t)i, t, lam, mu, sigma, NULL);
      neuron_step(m, NULL, n, i, m->C, V[i], p, ge[i], gi[i], I, &Vn, pn);
      s[i] = (uint8_t)(V[i] < m->v_th && Vn >= m->v_th);
      V[i] = Vn;
      for (int g = 0; g < G; ++g) state[(int64_t)(1 + g) * n + i] = pn[g];
    }
    /* a spike of step t through a synapse of delay d arrives at step t + d:
     * sources in index order, each row in CSR order */
    for (int64_t j = 0; j < n; ++j) {
      if (!s[j]) continue;
      for (int64_t e = row_ptr[j]; e < row_ptr[j + 1]; ++e) {
        const int64_t slot = (t + (delay ? delay[e] : 1)) % R;
        if (w[e] > 0.0) pend_e[slot * n + col[e]] += w_scale * w[e];
        else if (w[e] < 0.0) pend_i[slot * n + col[e]] += w_scale * (-w[e]);
      }
    }
    const int64_t a = (t + 1) % R;
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
    for (int64_t i = 0; i < n; ++i) {
      double ext = 0.0;
      if (ext_mask && ext_mask[i] && ora_event_word(seed, (uint32_t)i, t + 1) < ext_thresh)
        ext = w_ext;
      ge[i] = ge[i] * de + pend_e[a * n + i] + ext;
      gi[i] = gi[i] * di + pend_i[a * n + i];
      pend_e[a * n + i] = 0.0;
      pend_i[a * n + i] = 0.0;
      if (spk) spk[(int64_t)k * n + i] = s[i];
    }
  }
  free(s); free(pend_e); free(pend_i);
  return 0;
}

/* ---------------------------------------------------------------------------
 * Backpropagation through time of the discrete map (Methods, "Gradient
 * learning support"): the loss gradient is carried backwards through the
 * transposed Jacobian of each step, lambda_t = J_t^T lambda_{t+1} + dL/dx_t.
 * All Jacobian entries are closed form in the rate functions and their
 * derivatives.  Neurons are independent, so each is processed alone.
 * ------------------------------------------------------------------------- */
static double sigm(double x) { return 1.0 / (1.0 + exp(-x)); }

int32_t ora_bptt(const ora_model* m, int64_t n, const double* cm, const double* state0,
                 int32_t T, const double* I, const double* dL_dr, const double* dL_dV,
                 int32_t smooth, double beta, double* r_out, double* dI, double* dCm,
                 double* dx0) {
  if (!model_ok(m) || m->has_syn || m->tab_n != 0 || n < 0 || T <= 0) return -1;
  const int G = m->n_gates, NS = 1 + G;
  const double dt = m->dt, th = m->v_th;
  double* traj = (double*)malloc(sizeof(double) * (size_t)(T + 1) * NS);
  if (!traj) return -2;
  for (int64_t i = 0; i < n; ++i) {
    const double C = cm ? cm[i] : m->C;
    /* forward, keeping the whole trajectory of this neuron */
    for (int s = 0; s < NS; ++s) traj[s] = state0[(int64_t)s * n + i];
    double r = 0.0;
    for (int32_t t = 0; t < T; ++t) {
      const double* x = traj + (size_t)t * NS;
      double* xn = traj + (size_t)(t + 1) * NS;
      neuron_step(m, NULL, n, i, C, x[0], x + 1, 0.0, 0.0, I[(int64_t)t * n + i], &xn[0], xn + 1);
      double Vn = xn[0];
      r += smooth ? sigm(beta * (Vn - th)) : (Vn >= th ? 1.0 : 0.0);
    }
    r /= (double)T;
    if (r_out) r_out[i] = r;
    /* reverse sweep */
    double lam[1 + ORA_MAX_GATES], nl[1 + ORA_MAX_GATES];
    for (int s = 0; s < NS; ++s) lam[s] = 0.0;
    double dc = 0.0;
    for (int32_t t = T - 1; t >= 0; --t) {
      /* direct loss on x_{t+1}: only through V_{t+1} */
      double Vn = traj[(size_t)(t + 1) * NS];
      double sg = sigm(beta * (Vn - th));
      double dsdv = beta * sg * (1.0 - sg); /* surrogate / smooth derivative */
      if (dL_dr) lam[0] += dL_dr[i] * dsdv / (double)T;
      if (dL_dV) lam[0] += dL_dV[(int64_t)t * n + i];
      /* Jacobian of step t at x_t */
      const double* x = traj + (size_t)t * NS;
      const double V = x[0];
      const double* p = x + 1;
      const double It = I[(int64_t)t * n + i];
      double e[ORA_MAX_GATES], dpv[ORA_MAX_GATES]; /* dp'/dp, dp'/dV */
      for (int g = 0; g < G; ++g) {
        double pinf, eg, dpinf, deg;
        gate_terms(m, NULL, n, i, g, V, &pinf, &eg, &dpinf, &deg);
        e[g] = eg;
        dpv[g] = dpinf * (1.0 - eg) + (p[g] - pinf) * deg;
      }
      double dvdv, dvdI, dvdC, dvdp[ORA_MAX_GATES];
      double gsum = 0.0, nsum = 0.0, i_ion = 0.0, a[ORA_MAX_GATES], b[ORA_MAX_GATES];
      for (int g = 0; g < G; ++g) a[g] = b[g] = 0.0;
      for (int c = 0; c < m->n_channels; ++c) {
        double deta[ORA_MAX_GATES];
        double gx = m->ch_gbar[c] * channel_eta(m, c, p, deta);
        gsum += gx;
        nsum += gx * m->ch_E[c];
        i_ion += gx * (V - m->ch_E[c]);
        for (int g = 0; g < G; ++g) {
          a[g] += m->ch_gbar[c] * deta[g];                  /* d gtot / d p_g      */
          b[g] += m->ch_gbar[c] * deta[g] * (V - m->ch_E[c]); /* d I_ion / d p_g   */
        }
      }
      if (m->v_method == ORA_FE) {
        dvdv = 1.0 - (dt / C) * gsum;
        dvdI = dt / C;
        dvdC = -(dt / (C * C)) * (It - i_ion);
        for (int g = 0; g < G; ++g) dvdp[g] = -(dt / C) * b[g];
      } else {
        double num = It + nsum, vinf = num / gsum, E = exp(-dt * gsum / C);
        dvdv = E;
        dvdI = (1.0 - E) / gsum;
        dvdC = (V - vinf) * (dt * gsum / (C * C)) * E;
        for (int g = 0; g < G; ++g) {
          /* d num / d p_g = sum_X gbar deta E_X = a_g V - b_g */
          double dnum = a[g] * V - b[g];
          double dvinf = (dnum - vinf * a[g]) / gsum;
          double dE = -(dt / C) * a[g] * E;
          dvdp[g] = dvinf * (1.0 - E) + (V - vinf) * dE;
        }
      }
      if (dI) dI[(int64_t)t * n + i] = lam[0] * dvdI;
      dc += lam[0] * dvdC;
      nl[0] = lam[0] * dvdv;
      for (int g = 0; g < G; ++g) {
        nl[0] += lam[1 + g] * dpv[g];
        nl[1 + g] = lam[0] * dvdp[g] + lam[1 + g] * e[g];
      }
      for (int s = 0; s < NS; ++s) lam[s] = nl[s];
    }
    if (dCm) dCm[i] = dc;
    if (dx0)
      for (int s = 0; s < NS; ++s) dx0[(int64_t)s * n + i] = lam[s];
  }
  free(traj);
  return 0;
}
