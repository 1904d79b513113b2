/*
 * hh.h -- C ABI of libhh, an MI355X (gfx950) library that time-steps large
 * populations of Hodgkin-Huxley neurons with user-defined ion channels, and
 * differentiates through them.
 *
 * The model is the point-neuron form of the paper's Eq. (1) (Methods,
 * "Membrane potential and ion-channel definitions"):
 *     C dV/dt = I - sum_X gbar_X eta_X(p) (V - E_X) - I_syn,
 *     dp/dt   = alpha_p(V) (1 - p) - beta_p(V) p,
 * with eta_X a product of integer powers of gate variables, discretized as in
 * Methods, "Simplified discretization": exponential Euler for every gate,
 * explicit Euler for V (Eq. (2)) or exponential Euler in V.  All right-hand
 * sides of one step are evaluated at the state at the start of that step.
 * Channels are user-defined as a conductance plus activation/deactivation
 * rate terms ("Flexibility and extensibility").
 *
 * Conventions
 *  - All array arguments are DEVICE pointers unless marked (host).  The caller
 *    owns every buffer; the library owns only the opaque hh_model.
 *  - Layouts are structure-of-arrays.  A population has n = N * B neurons:
 *    B independent copies (a batch) of N neurons; neuron index b*N + i.
 *    Per-neuron parameters are [N] arrays shared across the batch.
 *  - A state buffer is float [n_state][n] with n_state = 2 + n_gates
 *    (+2 when the model has conductance synapses): V, then the gates in
 *    descriptor order, then g_e, g_i, and last V_lo.  The membrane potential
 *    is carried as the unevaluated sum V + V_lo of two floats so that
 *    per-step changes below half an FP32 ulp of V are not rounded away; V
 *    alone is the potential to FP32 precision.
 *  - Every call is asynchronous on `stream` (a hipStream_t; NULL = the null
 *    stream) except hh_init, hh_destroy and hh_check.
 *  - Return value: HH_OK, or a negative hh_status.  On any status other than
 *    HH_E_HIP nothing was launched.  No exceptions cross the ABI.
 *  - Calls that share one hh_model must not run concurrently on different
 *    streams (the model's small scratch buffers are reused).
 */
#ifndef HH_H
#define HH_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HH_MAX_GATES 8
#define HH_MAX_CHANNELS 8
#define HH_MAX_CH_GATES 4

typedef enum {
  HH_OK = 0,
  HH_E_INVALID = -1,     /* malformed descriptor or argument */
  HH_E_SHAPE = -2,       /* sizes inconsistent or out of range */
  HH_E_HIP = -3,         /* a HIP runtime call failed */
  HH_E_NONFINITE = -4,   /* hh_check: a state value became NaN/Inf */
  HH_E_UNSUPPORTED = -5, /* valid request the library does not implement */
  HH_E_OOM = -6,         /* the library could not allocate its own scratch */
  HH_E_TIMEOUT = -7      /* hh_check: a persistent kernel gave up waiting */
} hh_status;

/* Rate-function forms, u = (V - B) / K (V in mV, rates in 1/ms):
 *   HH_FORM_EXP      A e^u
 *   HH_FORM_SIGMOID  A / (1 + e^u)
 *   HH_FORM_LINOID   A (V - B) / (1 - e^{-u})        (value A K at V = B)
 *   HH_FORM_BELL     (c e^u + e^{-u}) / A                                   */
enum { HH_FORM_EXP = 0, HH_FORM_SIGMOID = 1, HH_FORM_LINOID = 2, HH_FORM_BELL = 3 };
/* A gate carries either the (alpha, beta) rates of Eq. (1) or (p_inf, 1/tau). */
enum { HH_GATE_ALPHA_BETA = 0, HH_GATE_INF_TAU = 1 };
/* Membrane update: explicit Euler (Eq. (2)) or exponential Euler in V. */
enum { HH_V_FE = 0, HH_V_EE = 1 };
/* External current. */
enum { HH_IN_NONE = 0, HH_IN_CONST = 1, HH_IN_NOISE = 2, HH_IN_DENSE = 3, HH_IN_BACKGROUND = 4,
       HH_IN_SINE = 5 };

typedef struct {
  int32_t form;
  float A, B, K, c;
} hh_rate;

typedef struct {
  int32_t kind;    /* HH_GATE_* */
  hh_rate r[2];    /* (alpha, beta) or (p_inf, 1/tau) */
} hh_gate;

typedef struct {
  float gbar, E;                 /* mS/cm^2, mV */
  int32_t n_gates;               /* 0..HH_MAX_CH_GATES factors; 0 = leak */
  int32_t gate[HH_MAX_CH_GATES]; /* gate index of each factor */
  int32_t expo[HH_MAX_CH_GATES]; /* integer exponent 0..8 */
} hh_channel;

typedef struct {
  int32_t n_gates, n_channels;
  hh_gate gates[HH_MAX_GATES];
  hh_channel channels[HH_MAX_CHANNELS];
  float C_m;      /* uF/cm^2 (used when no per-neuron C_m is given) */
  float dt;       /* ms */
  float v_th;     /* spike threshold, mV: a spike is an upward crossing */
  int32_t v_method;
  int32_t has_syn;             /* exponential-decay conductance synapses */
  float tau_e, tau_i, E_e, E_i;
} hh_model_desc;

typedef struct hh_model hh_model;

/* Input current for hh_step_n / hh_backward. */
typedef struct {
  int32_t mode;          /* HH_IN_* */
  const float* i_const;  /* HH_IN_CONST: [n] uA/cm^2 */
  float mu, sigma;       /* HH_IN_NOISE: I = mu + sigma z, z standard normal */
  uint64_t seed;         /* HH_IN_NOISE: Philox4x32-10 key */
  const float* i_dense;  /* HH_IN_DENSE: [n_steps][n], row t is step t0 + t */
  float lam;             /* HH_IN_BACKGROUND: expected events per step, [0, 80] */
  const float* freq;     /* HH_IN_SINE: [n] frequencies in Hz, 0 <= f <= 1000 / dt;
                            i_const then holds the [n] amplitudes */
} hh_input;
/* HH_IN_SINE (Results, HH encryption: sine-driven neurons): I = A sin(2 pi phi)
 * with phi the phase in revolutions.  The frequency is quantized to
 * R = round(f K) / 2^32 revolutions per step, f K taken in binary32 with
 * K = binary32(dt 2^32 / 1000), and the phase at absolute step t is exactly
 * (R t mod 2^32) / 2^32, so long runs accumulate no phase error. */
/* HH_IN_BACKGROUND (Methods, cortical network: the background input drawn
 * directly from its distribution): per element and step, N ~ Poisson(lam)
 * background events of independent Gaussian amplitude (mu, sigma), so
 * I = N mu + sqrt(N) sigma z.  The random words are Philox4x32-10 block
 * (t, stream 2) of the element, keyed by seed: word 0 gives
 * u = (2 floor(w0 / 2^9) + 1) 2^-24 and N is the smallest k with u <= F(k),
 * F the Poisson CDF accumulated in binary32 from p_0 = e^-lam (rounded once
 * from binary64) with each product, quotient and sum rounded on its own,
 * up to floor(lam + 12 sqrt(lam)) + 12; words 2 and 3 give z by Box-Muller
 * (cosine branch, u = (w + 1/2) 2^-32). */

/* Optional outputs of hh_step_n (any pointer may be NULL). */
typedef struct {
  uint32_t* spikes;   /* [n_steps][ceil(n/32)] bit i%32 of word i/32 = crossing */
  float* v_rec;       /* [n_steps][n] V after each step */
  float* ckpt;        /* [ceil(n_steps/ckpt_every)][n_state][n] state before
                         steps 0, ckpt_every, 2*ckpt_every, ... of this call */
  int32_t ckpt_every;
  float* level;       /* [n] += number of steps ending with V >= v_th */
} hh_outputs;

/* Create a model for n = N * B neurons from a host descriptor (copied)
 * (Methods, "Membrane potential and ion-channel definitions", Eq. (1): the
 * state is V and the gate variables p; the parameters are C_m and, per
 * channel X, gbar_X, E_X and the gates whose powers form eta_X(p); each gate
 * carries its alpha_p / beta_p rate functions.  "Flexibility and
 * extensibility": a channel is user-defined as a conductance plus its
 * activation and deactivation terms, here parameterized rate forms.  The B
 * copies are the paper's parallel simulations on one device (Results,
 * "Cortical scale: cortex simulation").)
 * coef: nullable [n_gates*8][N] per-neuron rate coefficients, row
 * g*8 + r*4 + j holding (A, B, K, c)[j] of rate r of gate g; replaces the
 * descriptor's values.  cm: nullable [N] per-neuron C_m.  Both stay owned by
 * the caller and must outlive the model.  Errors: HH_E_INVALID for a bad
 * descriptor (unknown form/kind, gate index out of range, dt <= 0, C_m <= 0,
 * tau <= 0), HH_E_SHAPE for N < 1, B < 1 or n >= 2^31. */
int32_t hh_init(hh_model** out, const hh_model_desc* desc, int64_t N, int32_t B,
                const float* coef, const float* cm);
int32_t hh_destroy(hh_model* m);
const char* hh_status_string(int32_t status);
int32_t hh_n_state(const hh_model* m);

/* Fusion depth: the number of steps one kernel launch keeps in registers
 * (Methods, "Engineering optimization": operator fusion).  Default 32. */
int32_t hh_set_fusion(hh_model* m, int32_t k_steps);

/* Channel sets whose structure (forms, gate kinds, exponents) matches one of
 * the library's compiled specializations -- the Hodgkin-Huxley (1952) set
 * and the cortical Na/Kd/M/L-Ca/leak set -- run straight-line kernels; any
 * other set runs the general interpreter.  on = 0 forces the interpreter
 * (results are identical up to FP32 rounding order).  Default 1. */
int32_t hh_set_specialize(hh_model* m, int32_t on);

/* Tabulated gate kinetics, an approximation of the rate functions (Methods,
 * "Engineering optimization": the rates' cost is cut by cheaper
 * approximations).  The gate update p' = p + (p_inf - p) q, q = 1 - e
 * (exponential Euler, "Simplified discretization") then takes p_inf(V) and
 * q(V) by linear interpolation between n_nodes equally spaced voltages from
 * v_lo to v_hi (mV), tabulated once on the device from the model's rate
 * functions in binary64 (q = -expm1(-dt (alpha + beta)), without
 * cancellation) and rounded once per entry; V outside [v_lo, v_hi] is
 * clamped to the range.  The membrane update is unchanged.  The table (n_gates x n_nodes x
 * 16 bytes) is owned by the model and used by every later hh_step_n;
 * n_nodes = 0 removes it.  Errors: HH_E_SHAPE for n_nodes outside [2, 2^20];
 * HH_E_INVALID for v_hi <= v_lo or non-finite bounds; HH_E_UNSUPPORTED unless
 * the channel set is one of the compiled ones (hh_set_specialize on), the
 * coefficients are uniform (no per-neuron table) and no network is attached.
 * Multi-compartment neurons (hh_set_morphology) use the table too.
 * hh_backward, hh_surrogate_step_n and the network path return
 * HH_E_UNSUPPORTED while a table is set (they evaluate the rate functions). */
int32_t hh_set_rate_table(hh_model* m, float v_lo, float v_hi, int32_t n_nodes, void* stream);

/* Multi-compartment neurons (Methods, Eq. (1) with its spatial term
 * (1/r_l) d2V/dx2; "Simplified discretization": the second-order explicit
 * difference in space).  Every neuron of the population becomes K
 * consecutive compartments: compartment c of neuron j is element j*K + c of
 * the population (and of every state row, input and output), so n = N*B
 * counts compartments and N must be a multiple of K.  All neurons share the
 * morphology, given as host arrays of K entries:
 *   parent[c]   the compartment c is attached to, in [0, c), or -1 for a
 *               root (a neuron may have several unconnected roots)
 *   g_axial[c]  the conductance of the edge c - parent[c] per unit of
 *               reference membrane area, mS/cm^2 (ignored for roots);
 *               nullable when K = 1
 *   area[c]     membrane area relative to the reference (nullable: all 1)
 *   gbar        nullable [K][n_channels]: the channel conductances of each
 *               compartment, replacing the descriptor's (passive dendrites,
 *               active soma, ...)
 * Each step, compartment c receives the axial current
 *     sum over its edges e of (g_e / area[c]) (V_other - V_c)
 * from the start-of-step potentials, added to its input current; for a
 * uniform unbranched cable with g = 1/(r_l dx^2) this is the central
 * difference (1/r_l)(V_{c-1} - 2V_c + V_{c+1})/dx^2 with sealed ends.
 * Explicit coupling is stable for dt * sum_e g_e / (C area) below about 1
 * (forward Euler).  K = 0 removes the morphology.  The arrays are copied;
 * the call returns when the copy is done.
 * Errors: HH_E_SHAPE for K not a power of two in [1, 64] or N not a multiple
 * of K; HH_E_INVALID for a parent outside [-1, c), a negative or non-finite
 * conductance, a non-positive area, or a missing array; HH_E_UNSUPPORTED for
 * more than 4 children on one compartment, or with a network attached.  A
 * rate table (hh_set_rate_table) applies to every compartment.  With a
 * morphology, hh_step_n refuses checkpoints, level counts and networks, and
 * hh_backward and hh_surrogate_step_n return HH_E_UNSUPPORTED. */
int32_t hh_set_morphology(hh_model* m, int32_t K, const int32_t* parent, const float* g_axial,
                          const float* area, const float* gbar, void* stream);

/* state <- (V0, p_inf(V0) for every gate, g_e = g_i = 0, V_lo = 0).  v0: nullable [n]
 * device array; when NULL every neuron starts at v0_scalar. */
int32_t hh_init_state(hh_model* m, float* state, const float* v0, float v0_scalar, void* stream);

/* Advance `state` by n_steps steps starting at absolute step t0 (the noise
 * generator is keyed by the absolute step, so runs can be split and resumed).
 * One step is Eq. (1) discretized as in Methods, "Simplified discretization":
 * every gate by exponential Euler, V by explicit Euler (Eq. (2), "Analysis of
 * C_m") or by exponential Euler, all right-hand sides at the start-of-step
 * state; a spike is the upward crossing of v_th within the step.  Many steps
 * are fused into one launch with the state in registers (Methods,
 * "Engineering optimization": operator fusion).
 * With a CSR attached (hh_attach_csr) the population is a recurrent network
 * and each step also delivers that step's spikes through the synapses.
 * Errors: HH_E_SHAPE for n_steps < 0 or ckpt_every < 1 with ckpt set;
 * HH_E_INVALID for a missing input array. */
int32_t hh_step_n(hh_model* m, float* state, int64_t t0, int32_t n_steps, const hh_input* in,
                  const hh_outputs* out, void* stream);

/* Synaptic connectivity for the recurrent network (Results, cortical network
 * with sparse synapses and indirect addressing): CSR by source neuron over
 * the N neurons of one copy, row_ptr int64 [N+1], col int32 [nnz] target ids
 * in [0, N), w float [nnz].  A spike of source j adds w_scale * w to g_e of
 * each target for w > 0 and w_scale * |w| to g_i for w < 0, one step after
 * the spike.  With B > 1 the population is B independent copies of the
 * network sharing this CSR (the paper's parallel simulations on one device,
 * Results, "Cortical scale: cortex simulation"): element b N + j spikes
 * through row j into targets b N + col.  hh_step_n runs all copies in one
 * co-resident grid and returns HH_E_UNSUPPORTED when N B neurons do not fit
 * one (two blocks of 512 per compute unit: 262,144 neurons on 256 compute
 * units).  When the rows list their targets in ascending order, the call
 * also builds a table of each row's offsets at every 512th target
 * (N (ceil(N / 512) + 1) int32, kept while it is no larger than the column
 * array), which the deliveries by target range use.  The call synchronizes
 * the device and reads the CSR once to check it.  Buffers stay owned by the
 * caller.  Requires has_syn.  Errors: HH_E_INVALID for missing arrays, a
 * negative or non-finite w_scale, or an invalid CSR (row_ptr not starting at
 * 0, decreasing, or not ending at nnz; a column outside [0, N)), in which
 * case the model keeps its previous connectivity; HH_E_SHAPE for nnz < 0;
 * HH_E_OOM; HH_E_HIP. */
int32_t hh_attach_csr(hh_model* m, const int64_t* row_ptr, const int32_t* col, const float* w,
                      int64_t nnz, float w_scale);

/* Delivery in the network time loop.  HH_DELIVERY_AUTO (the default): by
 * target range when the table of hh_attach_csr exists, the delays are one
 * step and either B = 1 or N >= 512 -- after each step's grid barrier every
 * block reads the lists of the previous step's spiking rows of the copies
 * its 512 elements belong to and adds their events for those elements in
 * on-chip memory; otherwise, and always with
 * HH_DELIVERY_PUSH, each spiking row is added into arrival accumulators by
 * device-scope atomics.  Both add the same 64-bit fixed-point increments,
 * so the results are identical.  Errors: HH_E_INVALID for another mode. */
enum { HH_DELIVERY_AUTO = 0, HH_DELIVERY_PUSH = 1 };
int32_t hh_set_delivery(hh_model* m, int32_t mode);
/* Synaptic delays of several steps (Methods, cortical network: per-pathway
 * synaptic delays): delay [nnz] (device, caller-owned, CSR order) gives each
 * synapse's delay in steps, in [1, max_delay] with max_delay <= 255; a spike
 * at step t then reaches g_e / g_i of its target at step t + delay instead
 * of t + 1.  A pathway delay is every synapse of the pathway carrying it.
 * The model keeps the arrivals still in flight in a ring of
 * (max_delay + 1) x 2 x n 64-bit accumulators: consecutive hh_step_n calls
 * on the same model (t0 continuing) deliver them, and a call with t0 = 0
 * starts with none in flight.  delay = NULL returns to one-step delays;
 * hh_attach_csr drops the table.  Errors: HH_E_INVALID without a CSR or for
 * a delay outside [1, max_delay] (the table is read back once to check);
 * HH_E_SHAPE for max_delay outside [1, 255]; HH_E_OOM. */
int32_t hh_set_delays(hh_model* m, const uint8_t* delay, int32_t max_delay);
/* External Poisson drive: neuron j of every copy with ext_mask[j] != 0
 * receives w_ext on g_e at step t when the stream-1 Philox4x32-10 word of
 * (seed, element index b N + j, t) is below thresh (event probability
 * thresh / 2^32 per step; each copy draws its own events).  ext_mask: device
 * [N], shared by the copies. */
int32_t hh_set_external(hh_model* m, const uint8_t* ext_mask, uint32_t thresh, float w_ext,
                        uint64_t seed);

/* One synaptic delivery outside the time loop (Results, "Practical deployment
 * on neuromorphic devices" and Methods, "Cerebral cortex network": spikes
 * delivered over sparse synapses by indirect addressing into conductance
 * synapses): compacts the spiking sources of `spike_bits` ([ceil(n/32)]
 * words) and adds their synaptic increments to g_e/g_i of `state`.  n_spikes_out: nullable device int32, receives the
 * number of spiking sources.  Accumulation is in 64-bit fixed point
 * (2^-40 mS/cm^2), so the result does not depend on the order of arrivals. */
int32_t hh_syn_propagate(hh_model* m, const uint32_t* spike_bits, float* state,
                         int32_t* n_spikes_out, void* stream);

/* Backpropagation through time (Methods, "Gradient learning support",
 * "Engineering optimization": manual gradients with re-computation).
 * Forward must have been run from step 0 with dense input and checkpoints
 * every ckpt_every steps (ckpt as written by hh_step_n).  The loss is
 *   L = sum_i dL_dlevel[i] * r_i + sum_{t,i} dL_dV[t][i] * V_{t+1,i},
 * r_i = (1/T) sum_{t=1..T} H(V_t - v_th), differentiated with the surrogate
 * dH/dV = beta s (1 - s), s = sigmoid(beta (V - v_th)).
 * Outputs: dI [T][n] = dL/dI_t (written), dCm [N] = dL/dC_m summed over the
 * batch (written; nullable), dx0 [n_state][n] (written; nullable).
 * workspace: device scratch of hh_backward_workspace() bytes.
 * Errors: HH_E_UNSUPPORTED for models with synapses or exponential Euler in
 * V; HH_E_SHAPE for T < 1 or ckpt_every < 1 or a short workspace. */
int32_t hh_backward(hh_model* m, const float* ckpt, int32_t ckpt_every, const hh_input* in,
                    int32_t T, const float* dL_dlevel, const float* dL_dV, float beta,
                    float* dI, float* dCm, float* dx0, void* workspace, size_t workspace_bytes,
                    void* stream);
/* The same adjoint over steps [t_lo, t_hi) only, so that work on the
 * gradients of later steps (dI rows t >= t_hi) can overlap the rest: calls
 * go from the end backwards over adjacent ranges (t_hi = T first, t_lo = 0
 * last), on one stream and one workspace, which carries the adjoint and the
 * dC_m partial sums between them.  t_lo and t_hi are multiples of ckpt_every
 * (t_hi may be T).  dI rows [t_lo, t_hi) are written; dCm and dx0 only by
 * the call with t_lo = 0.  hh_backward is the call with (0, T). */
int32_t hh_backward_part(hh_model* m, const float* ckpt, int32_t ckpt_every, const hh_input* in,
                         int32_t T, int32_t t_lo, int32_t t_hi, const float* dL_dlevel,
                         const float* dL_dV, float beta, float* dI, float* dCm, float* dx0,
                         void* workspace, size_t workspace_bytes, void* stream);
/* Bytes of the workspace of hh_backward / hh_backward_part for T steps with
 * checkpoints every ckpt_every steps: the adjoint carried between partial
 * calls, the dC_m partial sums, and the state at every 5th step of every
 * segment (recomputed from the segment's checkpoint by the call, for all of
 * its segments at once, before the reverse sweep): ceil(T / ckpt_every) x
 * ceil(ckpt_every / 5) x n_state x n floats when ckpt_every > 5.  0 for
 * invalid arguments. */
size_t hh_backward_workspace(const hh_model* m, int32_t ckpt_every, int32_t T);

/* Synchronize `stream` and report the first neuron whose state is not finite
 * (HH_E_NONFINITE, *first_bad = its index) or a persistent-kernel timeout
 * (HH_E_TIMEOUT).  Clears the flags. */
int32_t hh_check(hh_model* m, int64_t* first_bad, void* stream);

/* The output of the differentiable HH layer (Methods, "Gradient learning
 * support"; the rate that hh_backward differentiates): rate[i] = level[i] / T
 * for i < n, level as accumulated by hh_step_n over T steps (level and rate
 * may be the same array).  Errors: HH_E_INVALID for a NULL array,
 * HH_E_SHAPE for n < 0 or T < 1. */
int32_t hh_level_rate(const float* level, int64_t n, int32_t T, float* rate, void* stream);

/* Dense input projection of the layer in front of the neurons (the Linear
 * of the Sequential(Linear, HHNode) composition, Fig. 1e), on MFMA:
 *   out[M][N] (float) = A[M][K] (bf16) x Wt[N][K]^T (bf16), fp32 accumulate.
 * The weights are stored transposed (Wt [N][K], K contiguous), so that both
 * operands are K-contiguous.  All arrays row-major, device memory. */
int32_t hh_proj_forward(const uint16_t* A, const uint16_t* Wt, float* out, int32_t M, int32_t N,
                        int32_t K, void* stream);
/* The same product for a binary (spike) input given as bits:
 * A_bits [M][words_per_row] uint32 (device), bit k%32 of word k/32 of row m
 * is A[m][k] in {0, 1}; words_per_row >= ceil(K/32), bits at k >= K are
 * ignored.  A costs 1/16 of the bf16 input's memory traffic. */
int32_t hh_proj_forward_bits(const uint32_t* A_bits, int32_t words_per_row, const uint16_t* Wt,
                             float* out, int32_t M, int32_t N, int32_t K, void* stream);
/* Weight gradient dWt[N][K] = dOut^T A (float; written, or added to dWt's
 * contents when accumulate != 0, so a product over M can be split into
 * calls over row ranges), A [M][K] bf16, dOut [M][N] float (split into bf16
 * high and low parts inside the kernel, so the product keeps ~16 bits of
 * dOut).  The reduction over M is split into partial sums that are added in
 * a fixed order (bit-reproducible); workspace: device scratch of
 * hh_proj_wgrad_workspace(M, N, K) bytes (none for M == 0). */
int32_t hh_proj_wgrad(const uint16_t* A, const float* dOut, float* dWt, int32_t accumulate,
                      int32_t M, int32_t N, int32_t K, void* workspace, size_t workspace_bytes,
                      void* stream);
size_t hh_proj_wgrad_workspace(int32_t M, int32_t N, int32_t K);
/* The same weight gradient for a binary A given as bits in groups of 32
 * rows: A_bits [ceil(M/32)][ld] uint32 (device), ld >= K; bit b of word
 * (w, k) is A[32 w + b][k] in {0, 1} (bits of rows >= M are ignored).  The
 * words of consecutive columns k are adjacent, which makes the kernel's reads
 * of the spike operand whole cache lines.  Same workspace. */
int32_t hh_proj_wgrad_bits(const uint32_t* A_bits, int32_t ld, const float* dOut, float* dWt,
                           int32_t accumulate, int32_t M, int32_t N, int32_t K, void* workspace,
                           size_t workspace_bytes, void* stream);

/* Linear readout of the mean spike level and cross-entropy loss, forward and
 * backward (the readout layer of the differentiable network, Methods
 * "Training and preprocessing").  r = level / T with level [B][H] the
 * per-neuron count of steps with V >= v_th; logits = r W + bias, W [H][C],
 * bias [C]; loss = mean over b of -log softmax(logits_b)[labels[b]], with
 * every labels[b] in [0, C) (device data, not checked: an out-of-range label
 * leaves that row's loss term undefined).
 * Writes loss [1], dlevel [B][H] = dL/dr (the gradient with respect to the
 * rate r, which is what hh_backward's dL_dlevel takes), dW [H][C], db [C]
 * and, when non-NULL, logits [B][C].  C <= 32 (else HH_E_UNSUPPORTED).
 * workspace: hh_readout_ce_workspace(B, C) bytes. */
int32_t hh_readout_ce(const float* level, int32_t T, const float* W, const float* bias,
                      const int32_t* labels, int32_t B, int32_t H, int32_t C, float* loss,
                      float* dlevel, float* dW, float* db, float* logits, void* workspace,
                      size_t workspace_bytes, void* stream);
size_t hh_readout_ce_workspace(int32_t B, int32_t C);
/* hh_readout_ce for callers that cannot allocate device memory (code under
 * HIP graph capture, tight training or serving loops, harnesses that forbid
 * hipMalloc): the same kernels and results, with the scratch (dz [B][C] and
 * the row losses [B]) in a static device array of
 * HH_READOUT_NOALLOC_MAX_FLOATS floats (1 MiB) that each GPU the library runs
 * on holds until the process ends.  The call allocates nothing.  All calls on
 * one GPU share that array, so calls that overlap on one GPU (several streams
 * or threads) race; calls in stream order do not.  Errors as hh_readout_ce,
 * and HH_E_SHAPE for B * (C + 1) > HH_READOUT_NOALLOC_MAX_FLOATS (nothing
 * launched). */
#define HH_READOUT_NOALLOC_MAX_FLOATS 262144
int32_t hh_readout_ce_noalloc(const float* level, int32_t T, const float* W, const float* bias,
                              const int32_t* labels, int32_t B, int32_t H, int32_t C, float* loss,
                              float* dlevel, float* dW, float* db, float* logits, void* stream);

/* One Adam update (Kingma & Ba, 2015), step counted from 1:
 *   m = b1 m + (1 - b1) g,  v = b2 v + (1 - b2) g^2,
 *   p -= lr (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps).
 * param_bf16: nullable [count], receives p rounded to bf16 (for weights that
 * feed the MFMA projection). */
int32_t hh_adam_step(float* param, const float* grad, float* m, float* v, int64_t count, float lr,
                     float beta1, float beta2, float eps, int32_t step, uint16_t* param_bf16,
                     void* stream);

/* ---------------------------------------------------------------------------
 * Learned k-step surrogate.  A multilayer perceptron 7 -> 64 -> 64 -> 6 maps
 * (V, m, h, n, p, q, mean input current over the k steps) to the state
 * change over k steps of the cortical channel set; the plain integrator
 * stays the fallback and the judge of its error.  The network is trained on
 * transitions of the plain kernel (the method's own trajectories) and stands
 * in for k plain steps where it is admissible (Methods, "Engineering
 * optimization": cheaper approximations of the costly update).
 *
 * Hidden activation (the same for both hidden layers; a network is used with
 * the activation it was trained with):
 *   HH_ACT_SILU       a sigmoid(a)
 *   HH_ACT_HARDSWISH  a clamp(a / 6 + 1/2, 0, 1), the piecewise-quadratic
 *                     form of SiLU (Howard et al., 2019), evaluated without
 *                     transcendental functions
 *
 * params: float [HH_MLP_NPARAM] = W1 [7][64], b1 [64], W2 [64][64], b2 [64],
 * W3 [64][6], b3 [6], W[k][j] connecting input k to output j.
 * norm: float [32], the feature normalization: input mean [0..6], input
 * standard deviation [8..14], output mean [16..21], output standard deviation
 * [24..29].  The network sees x_n = (x - mean) / std and predicts the
 * normalized change; every entry point takes raw samples, X [S][7] and
 * Y [S][6] (state change), and normalizes inside. */
#define HH_MLP_NPARAM 5062
enum { HH_ACT_SILU = 0, HH_ACT_HARDSWISH = 1 };

/* Training set from plain trajectories: traj [T][n_state][n] is the state
 * before every step (hh_step_n checkpoints with ckpt_every = 1; n_state = 7:
 * V, m, h, n, p, q, V_lo), i_dense [T][n] the input of every step.  Step t of
 * element i (t + k < T) gives a sample when V <= v_fb both before step t and
 * before step t + k (V = V + V_lo): X = (state at t, mean input over steps
 * t .. t + k - 1, summed in step order in binary32 and divided by k, as the
 * deployment forms it), Y = state at t + k minus state at t.  Samples are
 * written in (t, i) order up to cap; *count (device int64) receives the
 * number of qualifying samples (which may exceed cap).  workspace:
 * hh_surrogate_transitions_workspace(T, k) bytes.  Errors: HH_E_UNSUPPORTED
 * for n_state != 7; HH_E_SHAPE for k outside [1, T) or a short workspace. */
int32_t hh_surrogate_transitions(const float* traj, int32_t n_state, const float* i_dense,
                                 int64_t n, int32_t T, int32_t k, float v_fb, float* X, float* Y,
                                 int64_t cap, int64_t* count, void* workspace,
                                 size_t workspace_bytes, void* stream);
size_t hh_surrogate_transitions_workspace(int32_t T, int32_t k);

/* Feature normalization of a training set: norm (written, all 32 entries)
 * gets the mean and the sample standard deviation (denominator S - 1) of
 * each input and target feature, floored at 1e-6 (inputs) and 1e-9
 * (targets); binary64 sums in a fixed order.  workspace:
 * hh_mlp_norm_workspace() bytes. */
int32_t hh_mlp_norm(const float* X, const float* Y, int64_t S, float* norm, void* workspace,
                    size_t workspace_bytes, void* stream);
size_t hh_mlp_norm_workspace(void);

/* Mean-squared-error loss on the normalized targets,
 * L = (1/S) sum_s sum_o (y_so - Yn_so)^2, and its gradient with respect to
 * params (written).  quantize != 0 rounds the weights and hidden activations
 * to bf16 where the MFMA inference does (straight-through gradient).  Partial
 * sums are added in a fixed order.  workspace: hh_mlp_grad_workspace(S)
 * bytes.  loss: device float, nullable. */
int32_t hh_mlp_grad(const float* params, const float* norm, const float* X, const float* Y,
                    int32_t S, int32_t quantize, int32_t act, float* grad, float* loss,
                    void* workspace, size_t workspace_bytes, void* stream);
size_t hh_mlp_grad_workspace(int32_t S);
/* FP32 forward (VALU) on raw inputs: Y [S][6] = de-normalized outputs. */
int32_t hh_mlp_forward(const float* params, const float* norm, const float* X, int32_t S,
                       int32_t quantize, int32_t act, float* Y, void* stream);
/* Pack params into the bf16 MFMA fragment image used by hh_mlp_infer and
 * hh_surrogate_step_n, together with the normalization.  packed: device
 * buffer of hh_mlp_packed_bytes(). */
int32_t hh_mlp_pack(const float* params, const float* norm, void* packed, void* stream);
size_t hh_mlp_packed_bytes(void);
/* MFMA inference on raw inputs X [S][7]: Y [S][6] = de-normalized outputs
 * (state change). */
int32_t hh_mlp_infer(const void* packed, int32_t act, const float* X, int32_t S, float* Y,
                     void* stream);

/* Advance a population of the cortical channel set by n_steps (a multiple of
 * k) using the surrogate for k steps at a time where it is admissible:
 * a neuron uses the plain integrator for a call when V > v_fallback before
 * or after the surrogate step, when it failed the last periodic check, and on
 * every check_every-th call, where all neurons run the plain integrator and
 * |V_plain - V_surrogate| > check_tol marks a neuron plain until the next
 * check (check_every = 0 disables checks).  Spikes come from plain steps
 * only.  flags: device uint8 [n], per-neuron check state (caller zeroes it
 * before the first call).  spikes: nullable [n_steps][ceil(n/32)].
 * stats: nullable device uint64 [3], incremented by (surrogate calls, plain
 * calls, failed checks).  The model must be the cortical set without
 * per-neuron coefficients or capacitance (else HH_E_UNSUPPORTED); input
 * HH_IN_NOISE or HH_IN_DENSE. */
int32_t hh_surrogate_step_n(hh_model* m, const void* mlp_packed, int32_t act, float* state,
                            uint8_t* flags, int64_t t0, int32_t n_steps, int32_t k,
                            const hh_input* in, float v_fallback, int32_t check_every,
                            float check_tol, uint32_t* spikes, uint64_t* stats, void* stream);

#ifdef __cplusplus
}
#endif
#endif
