/*
 * hh_oracle.h -- FP64 reference integrator for Hodgkin-Huxley populations.
 *
 * TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test suite, the smoke entry
 * and the CPU-baseline leg of the benchmark load this library.  It shares no
 * code, header, table or constant with the HIP library: every formula here is
 * written out from the paper's model statement (Methods, "Membrane potential
 * and ion-channel definitions", Eq. (1); "Analysis of C_m", Eq. (2);
 * "Simplified discretization") and from the published definitions it names
 * (Philox4x32-10, Box-Muller).
 *
 * Everything is plain, single-threaded, double precision, evaluated in the
 * order the model defines it.  No blocking, fusion or reordering.
 */
#ifndef HH_ORACLE_H
#define HH_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORA_MAX_GATES 8
#define ORA_MAX_CH 8

/* Rate-function forms, u = (V - B) / K:
 *   ORA_EXP      A * exp(u)
 *   ORA_SIGMOID  A / (1 + exp(u))
 *   ORA_LINOID   A * (V - B) / (1 - exp(-u))          (limit A*K at V = B)
 *   ORA_BELL     (c * exp(u) + exp(-u)) / A                                    */
enum { ORA_EXP = 0, ORA_SIGMOID = 1, ORA_LINOID = 2, ORA_BELL = 3 };
/* Gate kinds: rate pair (alpha, beta) of Eq. (1), or (p_inf, 1/tau). */
enum { ORA_AB = 0, ORA_INFTAU = 1 };
/* Membrane update: explicit Euler of Eq. (2), or exponential Euler in V. */
enum { ORA_FE = 0, ORA_EE = 1 };
/* External current modes. */
enum { ORA_IN_NONE = 0, ORA_IN_CONST = 1, ORA_IN_NOISE = 2, ORA_IN_DENSE = 3, ORA_IN_BACKGROUND = 4,
       ORA_IN_SINE = 5 };

typedef struct {
  int32_t n_gates, n_channels, v_method, has_syn;
  int32_t gate_kind[ORA_MAX_GATES];
  int32_t rate_form[ORA_MAX_GATES][2];
  double rate_coef[ORA_MAX_GATES][2][4]; /* A, B, K, c */
  int32_t ch_n[ORA_MAX_CH];
  int32_t ch_gate[ORA_MAX_CH][4];
  int32_t ch_expo[ORA_MAX_CH][4];
  double ch_gbar[ORA_MAX_CH], ch_E[ORA_MAX_CH];
  double C, dt, v_th;
  double tau_e, tau_i, E_e, E_i;
  /* Tabulated gate kinetics (Methods, "Engineering optimization": cheaper
   * approximations of the rate functions).  tab_n = 0: the rate functions
   * themselves.  tab_n >= 2: nodes v_k = tab_vlo + k tab_h, k = 0..tab_n-1. */
  int32_t tab_n;
  double tab_vlo, tab_h;
} ora_model;

/* Per-neuron coefficient override: coef[(g*8 + r*4 + j) * n + i] replaces
 * rate_coef[g][r][j] for neuron i (nullable).  cm[i] replaces C (nullable). */

/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11). */
void ora_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* Standard normal for (seed, id, absolute step t): Box-Muller on the Philox
 * block (t >> 2); component t & 3. */
double ora_noise(uint64_t seed, uint32_t id, int64_t t);
/* Raw 32-bit event word for (seed, id, absolute step t), stream 1. */
uint32_t ora_event_word(uint64_t seed, uint32_t id, int64_t t);
/* Background input for (seed, id, absolute step t): N ~ Poisson(lam) events
 * of Gaussian amplitude (mu, sigma), returned as N mu + sqrt(N) sigma z;
 * count (nullable) receives N.  ora_background_count: N for Philox word w0
 * (inverse transform in binary32). */
int32_t ora_background_count(uint32_t w0, double lam);
/* Sinusoidal input (Results, HH encryption: sine-driven HH neurons):
 * amplitude amp (uA/cm^2), frequency f (Hz), step dt (ms).  The frequency
 * is quantized to R = round(f * K) revolutions / 2^32 per step, the product
 * f * K taken in binary32 with K = binary32(dt 2^32 / 1000); the phase of
 * absolute step t is (R t mod 2^32) / 2^32 revolutions, exactly. */
uint32_t ora_sine_rate(double f, double dt);
double ora_sine(double amp, uint32_t R, int64_t t);
double ora_background(uint64_t seed, uint32_t id, int64_t t, double lam, double mu, double sigma,
                      int32_t* count);

/* One rate function and its V-derivative. */
double ora_rate(int32_t form, const double k[4], double V, double* dV);
/* Steady state of gate g at V (p_inf). */
double ora_gate_inf(const ora_model* m, const double* coef, int64_t n, int64_t i,
                    int32_t g, double V);
/* The two terms of the exponential-Euler gate update p' = p + (P - p) Q:
 * P = p_inf(V), Q = 1 - exp(-dt / tau(V)).  With tab_n >= 2 both are the
 * straight-line interpolants between the two nodes around V (V clamped to
 * the node range) of the same terms evaluated at the nodes. */
void ora_gate_pq(const ora_model* m, const double* coef, int64_t n, int64_t i, int32_t g,
                 double V, double* P, double* Q);
/* state[0][i] = v0[i]; state[1+g][i] = p_inf(v0[i]); synaptic slots = 0. */
void ora_init_state(const ora_model* m, const double* coef, int64_t n, const double* v0,
                    double* state);
int32_t ora_n_state(const ora_model* m);

/* Independent neurons, T steps from absolute step t0.  state [n_state][n] is
 * advanced in place.  spk [T][n] gets 1 for an upward crossing of v_th,
 * vrec [T][n] the membrane potential after each step, level[i] += number of
 * steps with V >= v_th.  ids: global neuron ids for the noise generator
 * (nullable = 0..n-1).  Returns 0, or -1 on a malformed model. */
/* Threads the parallel loops use (1 in the serial build). */
int32_t ora_threads(void);
int32_t ora_run(const ora_model* m, int64_t n, const double* coef, const double* cm,
                const uint32_t* ids, double* state, int64_t t0, int32_t T, int32_t in_mode,
                const double* i_const, double mu, double sigma, uint64_t seed, double lam,
                const double* i_dense, uint8_t* spk, double* vrec, double* level);
/* ORA_IN_SINE for ora_run: i_const holds the amplitudes [n] and freq the
 * frequencies [n] (Hz); ora_run_sine is ora_run with that extra array. */
int32_t ora_run_sine(const ora_model* m, int64_t n, const double* coef, const double* cm,
                     double* state, int64_t t0, int32_t T, const double* amp, const double* freq,
                     uint8_t* spk, double* vrec, double* level);

/* Multi-compartment neurons: n = N*K compartments, compartment c of neuron j
 * at j*K + c; parent[c] in [-1, c); g_axial [K] edge conductances per unit
 * reference area; area [K] relative membrane areas (nullable: 1); gbar
 * [K][n_channels] per-compartment channel conductances (nullable); coef,
 * cm and ids per element as in ora_run (nullable).  Inputs, state and outputs as ora_run (noise ids = element
 * index).  Returns 0, or -1 on a malformed model or morphology. */
int32_t ora_cable_run(const ora_model* m, int64_t n, int32_t K, const int32_t* parent,
                      const double* g_axial, const double* area, const double* gbar,
                      const double* coef, const double* cm, const uint32_t* ids, double* state,
                      int64_t t0, int32_t T, int32_t in_mode, const double* i_const, double mu,
                      double sigma, uint64_t seed, double lam, const double* i_dense, uint8_t* spk,
                      double* vrec);

/* Recurrent network with exponential-decay conductance synapses.  delay
 * (nullable): per-synapse delays in steps, [nnz], each in [1, max_delay].
 * in_mode: ORA_IN_NONE, ORA_IN_CONST (i_const [n]) or ORA_IN_BACKGROUND
 * (lam, mu, sigma, in_seed). */
int32_t ora_net_run(const ora_model* m, int64_t n, double* state, const int64_t* row_ptr,
                    const int32_t* col, const double* w, double w_scale, const uint8_t* delay,
                    int32_t max_delay, const uint8_t* ext_mask, uint32_t ext_thresh, double w_ext,
                    uint64_t seed, int32_t in_mode, const double* i_const, double mu, double sigma,
                    uint64_t in_seed, double lam, int64_t t0, int32_t T, uint8_t* spk);

/* One synaptic delivery: g_e[i] += scale*w for every synapse j->i with w > 0
 * and s_j = 1; g_i[i] += scale*|w| for w < 0.  In CSR order. */
void ora_syn_deliver(int64_t n, const int64_t* row_ptr, const int32_t* col, const double* w,
                     double w_scale, const uint8_t* s, double* ge, double* gi);

/* Backpropagation through time of the discrete map.  Forward from state0 over
 * dense input I [T][n]; outputs r[i] = (1/T) sum_{t=1..T} s_t with s_t the
 * level H(V_t - v_th) (smooth = 0) or sigmoid(beta (V_t - v_th)) (smooth = 1).
 * Loss L = sum_i dL_dr[i] r[i] + sum_{t,i} dL_dV[t][i] V_{t+1}  (both
 * nullable; V_{t+1} is the potential after step t).  Gradients: dI [T][n],
 * dCm [n] (per neuron), dx0 [n_state][n]; any may be null. */
int32_t ora_bptt(const ora_model* m, int64_t n, const double* cm, const double* state0,
                 int32_t T, const double* I, const double* dL_dr, const double* dL_dV,
                 int32_t smooth, double beta, double* r_out, double* dI, double* dCm,
                 double* dx0);

#ifdef __cplusplus
}
#endif
#endif
