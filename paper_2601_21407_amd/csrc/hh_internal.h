// hh_internal.h -- host-side model object and kernel launchers of libhh.
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/hh.h"
#include "hh_device.h"

struct StepArgs {
  float* state;
  int64_t n, N;
  const float* coef;
  const float* cm;
  int64_t t0;
  int32_t nsteps, k_base;
  int32_t in_mode;
  const float* i_const;
  float mu, sigma;
  uint64_t seed;
  float bg_lam, bg_p0;   // background input: events per step, e^-lam
  int32_t bg_kmax;       // and the count's cap
  const float* freq;     // sinusoidal input: [n] Hz (amplitudes in i_const)
  float sine_K;          // dt 2^32 / 1000 in binary32
  const float* i_dense;  // row 0 = step k_base of the call
  uint32_t* spikes;      // row 0 = step k_base of the call
  int64_t words;
  float* v_rec;          // row 0 = step k_base of the call
  float* ckpt;           // slot 0 = step 0 of the call
  int32_t ckpt_every;
  float* level;
  int32_t* bad;
  // tabulated gate kinetics (null: the rate functions)
  const float4* tab;
  int32_t tab_n;
  float tab_vlo, tab_inv_h;
  // morphology: K compartments per neuron (a power of two up to 64), at
  // most D children per compartment
  const hhk::CableComp* cable;
  int32_t cable_K, cable_D;
};

struct hh_model {
  hh_model_desc desc;
  hhk::KModel km;
  int64_t N, n;
  int32_t B;
  const float* coef;
  const float* cm;
  int32_t k_fuse;
  int32_t use_fixed;  // launch compiled channel-set specializations when they match
  int device;
  // device flags: [0] first non-finite neuron (INT32_MAX = none), [1] timeout
  int32_t* d_flags;
  // recurrent network
  // deliveries by target range (rows sorted by target, one copy): for row j
  // and target range r (512 targets each, a network block's neurons),
  // d_seg[j (R + 1) + r] is the offset within the row of its first target
  // >= 512 r; null when the rows are not sorted, B > 1 or the table would
  // be larger than the column array
  int32_t* d_seg;
  int32_t seg_R;
  // network time loop: deliver by pull when the segment table exists (1,
  // the default) or always by push (0)
  int32_t net_pull;
  const int64_t* row_ptr;
  const int32_t* col;
  const float* w;
  int64_t nnz;
  float w_scale;
  const uint8_t* ext_mask;
  uint32_t ext_thresh;
  float w_ext;
  uint64_t ext_seed;
  // synaptic delays: per-synapse steps (caller-owned [nnz]) and the ring of
  // arrivals in flight, [max_delay + 1][2][n] (owned; null: one-step delay)
  const uint8_t* delay;
  int32_t max_delay;
  unsigned long long* d_ring;
  // scratch for synaptic delivery: int64 accumulators [2][2][n], spike list [n],
  // counters and the grid barrier
  void* d_scratch;
  size_t scratch_bytes;
  // tabulated gate kinetics, owned by the model (null: none)
  float4* d_tab;
  int32_t tab_n;
  // lookup u = (V - tab_vlo) * tab_inv_h; node i sits at tab_vlo + i / tab_inv_h
  float tab_vlo, tab_inv_h;
  // morphology (multi-compartment neurons), owned by the model (null: none)
  hhk::CableComp* d_cable;
  int32_t cable_K, cable_D;
  int32_t cable_gbar;  // per-compartment channel conductances given
};

// Dispatch on the channel-set structure: compiled specializations for the
// built-in sets, the run-time interpreter for any other set.
template <template <class> class F, class... Args>
inline hipError_t dispatch_spec(const hhk::KModel& km, bool allow_fixed, Args... args) {
  using namespace hhk;
  if (allow_fixed && ClassicSpec::matches(km)) return F<ClassicSpec>::run(args...);
  if (allow_fixed && CorticalSpec::matches(km)) return F<CorticalSpec>::run(args...);
  switch (km.n_gates) {
    case 0: return F<GenericSpec<0>>::run(args...);
    case 1: return F<GenericSpec<1>>::run(args...);
    case 2: return F<GenericSpec<2>>::run(args...);
    case 3: return F<GenericSpec<3>>::run(args...);
    case 4: return F<GenericSpec<4>>::run(args...);
    case 5: return F<GenericSpec<5>>::run(args...);
    case 6: return F<GenericSpec<6>>::run(args...);
    case 7: return F<GenericSpec<7>>::run(args...);
    default: return F<GenericSpec<8>>::run(args...);
  }
}

hipError_t launch_init_state(const hh_model* m, float* state, const float* v0, float v0s,
                             hipStream_t s);
hipError_t launch_step(const hh_model* m, const StepArgs& a, hipStream_t s);
// fills m->d_tab (m->tab_n nodes from m->tab_vlo, spacing 1 / m->tab_inv_h)
hipError_t launch_build_table(const hh_model* m, hipStream_t s);
// the step of multi-compartment neurons (hh_cable.hip): a.cable set
hipError_t launch_cable(const hh_model* m, const StepArgs& a, hipStream_t s);

// recurrent network path of hh_step_n (hh_net.hip)
int32_t hh_net_step_n_internal(hh_model* m, float* state, int64_t t0, int32_t n_steps,
                               const hh_input* in, const hh_outputs* out, void* stream);
