// hh_api.cpp -- C ABI of libhh: argument validation, model set-up and
// launch planning.  No computation of the method happens here; every step of
// the path runs in the HIP kernels.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <new>

#include "hh_internal.h"

using namespace hhk;

#define HIP_OK(x)                        \
  do {                                   \
    if ((x) != hipSuccess) return HH_E_HIP; \
  } while (0)

static int valid_rate(const hh_rate& r) {
  if (r.form < HH_FORM_EXP || r.form > HH_FORM_BELL) return 0;
  if (!(r.K != 0.0f) || !isfinite(r.K) || !isfinite(r.A) || !isfinite(r.B) || !isfinite(r.c))
    return 0;
  if (r.form == HH_FORM_BELL && r.A == 0.0f) return 0;
  return 1;
}

static int validate_desc(const hh_model_desc* d) {
  if (!d) return 0;
  if (d->n_gates < 0 || d->n_gates > HH_MAX_GATES) return 0;
  if (d->n_channels < 0 || d->n_channels > HH_MAX_CHANNELS) return 0;
  for (int g = 0; g < d->n_gates; ++g) {
    const hh_gate& G = d->gates[g];
    if (G.kind != HH_GATE_ALPHA_BETA && G.kind != HH_GATE_INF_TAU) return 0;
    if (!valid_rate(G.r[0]) || !valid_rate(G.r[1])) return 0;
  }
  for (int c = 0; c < d->n_channels; ++c) {
    const hh_channel& C = d->channels[c];
    if (C.n_gates < 0 || C.n_gates > HH_MAX_CH_GATES) return 0;
    if (!isfinite(C.gbar) || !isfinite(C.E)) return 0;
    for (int k = 0; k < C.n_gates; ++k) {
      if (C.gate[k] < 0 || C.gate[k] >= d->n_gates) return 0;
      if (C.expo[k] < 0 || C.expo[k] > 8) return 0;
    }
  }
  if (!(d->dt > 0.0f) || !(d->C_m > 0.0f) || !isfinite(d->v_th)) return 0;
  if (d->v_method != HH_V_FE && d->v_method != HH_V_EE) return 0;
  if (d->has_syn && (!(d->tau_e > 0.0f) || !(d->tau_i > 0.0f))) return 0;
  return 1;
}

// Derived per-rate constants (see KRate), in double then rounded once.
static KRate derive_host(const hh_rate& r) {
  const double l2e = 1.4426950408889634;
  KRate k;
  const double s = l2e / r.K;
  k.s = (float)s;
  k.o = (float)(-(double)r.B * s);
  k.c = r.c;
  k.ik = (float)(1.0 / r.K);
  if (r.form == HH_FORM_LINOID) k.a = (float)((double)r.A * r.K);
  else if (r.form == HH_FORM_BELL) k.a = (float)(1.0 / r.A);
  else k.a = r.A;
  return k;
}

static void build_kmodel(const hh_model_desc* d, KModel* k) {
  memset(k, 0, sizeof(*k));
  k->n_gates = d->n_gates;
  k->n_ch = d->n_channels;
  k->v_method = d->v_method;
  k->has_syn = d->has_syn ? 1 : 0;
  for (int g = 0; g < d->n_gates; ++g) {
    k->kind[g] = d->gates[g].kind;
    for (int r = 0; r < 2; ++r) {
      k->form[g][r] = d->gates[g].r[r].form;
      k->rate[g][r] = derive_host(d->gates[g].r[r]);
    }
  }
  for (int c = 0; c < d->n_channels; ++c) {
    k->gbar[c] = d->channels[c].gbar;
    k->E[c] = d->channels[c].E;
    for (int q = 0; q < d->channels[c].n_gates; ++q)
      k->cexp[c][d->channels[c].gate[q]] += d->channels[c].expo[q];
  }
  k->dt = d->dt;
  k->v_th = d->v_th;
  k->C = d->C_m;
  k->kdt = (float)(-(double)d->dt * 1.4426950408889634);
  if (d->has_syn) {
    k->decay_e = (float)exp(-(double)d->dt / d->tau_e);
    k->decay_i = (float)exp(-(double)d->dt / d->tau_i);
    k->E_e = d->E_e;
    k->E_i = d->E_i;
  } else {
    k->decay_e = k->decay_i = 1.0f;
  }
}

extern "C" {

const char* hh_status_string(int32_t s) {
  switch (s) {
    case HH_OK: return "ok";
    case HH_E_INVALID: return "invalid argument or descriptor";
    case HH_E_SHAPE: return "inconsistent or out-of-range sizes";
    case HH_E_HIP: return "HIP runtime error";
    case HH_E_NONFINITE: return "non-finite state";
    case HH_E_UNSUPPORTED: return "unsupported request";
    case HH_E_OOM: return "out of device memory";
    case HH_E_TIMEOUT: return "persistent kernel timed out";
    default: return "unknown status";
  }
}

int32_t hh_init(hh_model** out, const hh_model_desc* desc, int64_t N, int32_t B,
                const float* coef, const float* cm) {
  if (!out) return HH_E_INVALID;
  *out = nullptr;
  if (!validate_desc(desc)) return HH_E_INVALID;
  if (N < 1 || B < 1) return HH_E_SHAPE;
  const int64_t n = N * (int64_t)B;
  if (n >= ((int64_t)1 << 31)) return HH_E_SHAPE;
  hh_model* m = new (std::nothrow) hh_model();
  if (!m) return HH_E_OOM;
  m->desc = *desc;
  build_kmodel(desc, &m->km);
  m->N = N;
  m->B = B;
  m->n = n;
  m->coef = coef;
  m->cm = cm;
  m->k_fuse = 32;
  m->use_fixed = 1;
  m->net_pull = 1;
  if (hipGetDevice(&m->device) != hipSuccess) {
    delete m;
    return HH_E_HIP;
  }
  if (hipMalloc((void**)&m->d_flags, 4 * sizeof(int32_t)) != hipSuccess) {
    delete m;
    return HH_E_OOM;
  }
  const int32_t init_flags[4] = {INT32_MAX, 0, 0, 0};
  if (hipMemcpy(m->d_flags, init_flags, sizeof(init_flags), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(m->d_flags);
    delete m;
    return HH_E_HIP;
  }
  *out = m;
  return HH_OK;
}

int32_t hh_destroy(hh_model* m) {
  if (!m) return HH_OK;
  if (m->d_tab) (void)hipFree(m->d_tab);
  if (m->d_cable) (void)hipFree(m->d_cable);
  if (m->d_ring) (void)hipFree(m->d_ring);
  if (m->d_scratch) (void)hipFree(m->d_scratch);
  if (m->d_seg) (void)hipFree(m->d_seg);
  if (m->d_flags) (void)hipFree(m->d_flags);
  delete m;
  return HH_OK;
}

int32_t hh_n_state(const hh_model* m) {
  if (!m) return HH_E_INVALID;
  return 2 + m->km.n_gates + (m->km.has_syn ? 2 : 0);
}

int32_t hh_set_fusion(hh_model* m, int32_t k) {
  if (!m) return HH_E_INVALID;
  if (k < 1) return HH_E_SHAPE;
  m->k_fuse = k;
  return HH_OK;
}

int32_t hh_set_specialize(hh_model* m, int32_t on) {
  if (!m) return HH_E_INVALID;
  m->use_fixed = on ? 1 : 0;
  return HH_OK;
}

int32_t hh_set_morphology(hh_model* m, int32_t K, const int32_t* parent, const float* g_axial,
                          const float* area, const float* gbar, void* stream) {
  if (!m) return HH_E_INVALID;
  hipStream_t s = (hipStream_t)stream;
  if (K == 0) {
    if (m->d_cable) {
      HIP_OK(hipStreamSynchronize(s));
      HIP_OK(hipFree(m->d_cable));
    }
    m->d_cable = nullptr;
    m->cable_K = m->cable_D = m->cable_gbar = 0;
    return HH_OK;
  }
  if (K < 1 || K > 64 || (K & (K - 1)) != 0 || m->N % K != 0) return HH_E_SHAPE;
  if (!parent || (K > 1 && !g_axial)) return HH_E_INVALID;
  if (m->row_ptr) return HH_E_UNSUPPORTED;
  const int nch = m->km.n_ch;
  hhk::CableComp comp[64];
  int nchild[64];
  memset(comp, 0, sizeof(comp));
  for (int c = 0; c < K; ++c) {
    const int p = parent[c];
    if (p < -1 || p >= c) return HH_E_INVALID;  // roots, or an earlier compartment
    const float a = area ? area[c] : 1.0f;
    if (!(a > 0.0f) || !(a < 1e30f)) return HH_E_INVALID;
    if (p >= 0 && (!(g_axial[c] >= 0.0f) || !(g_axial[c] < 1e30f))) return HH_E_INVALID;
    comp[c].par = c;
    for (int d = 0; d < hhk::kMaxChildren; ++d) comp[c].ch[d] = c;
    nchild[c] = 0;
    for (int x = 0; x < hhk::kMaxCh; ++x) {
      float g = x < nch ? m->km.gbar[x] : 0.0f;
      if (gbar && x < nch) {
        g = gbar[(int64_t)c * nch + x];
        if (!(g >= 0.0f) || !(g < 1e30f)) return HH_E_INVALID;
      }
      comp[c].gbar[x] = g;
    }
  }
  int D = 0;
  for (int c = 0; c < K; ++c) {
    const int p = parent[c];
    if (p < 0) continue;
    const float g = g_axial[c];
    comp[c].par = p;
    comp[c].gup = g / (area ? area[c] : 1.0f);
    const int d = nchild[p]++;
    if (d >= hhk::kMaxChildren) return HH_E_UNSUPPORTED;
    comp[p].ch[d] = c;
    comp[p].gdn[d] = g / (area ? area[p] : 1.0f);
    if (d + 1 > D) D = d + 1;
  }
  if (!m->d_cable && hipMalloc((void**)&m->d_cable, sizeof(comp)) != hipSuccess) {
    m->d_cable = nullptr;
    return HH_E_OOM;
  }
  HIP_OK(hipMemcpyAsync(m->d_cable, comp, sizeof(comp), hipMemcpyHostToDevice, s));
  HIP_OK(hipStreamSynchronize(s));  // comp lives on this stack frame
  m->cable_K = K;
  m->cable_D = D;
  m->cable_gbar = gbar ? 1 : 0;
  return HH_OK;
}

int32_t hh_set_rate_table(hh_model* m, float v_lo, float v_hi, int32_t n_nodes, void* stream) {
  if (!m) return HH_E_INVALID;
  if (n_nodes == 0) {
    if (m->d_tab) {
      HIP_OK(hipStreamSynchronize((hipStream_t)stream));
      HIP_OK(hipFree(m->d_tab));
    }
    m->d_tab = nullptr;
    m->tab_n = 0;
    return HH_OK;
  }
  if (n_nodes < 2 || n_nodes > (1 << 20)) return HH_E_SHAPE;
  if (!(v_hi > v_lo) || !(fabsf(v_lo) < 1e30f) || !(fabsf(v_hi) < 1e30f)) return HH_E_INVALID;
  // the tabulated step exists for the built-in channel sets with uniform
  // coefficients, outside the network (the network, adjoint and surrogate
  // kernels evaluate the rate functions)
  if (m->coef || m->row_ptr || !m->use_fixed) return HH_E_UNSUPPORTED;
  if (!(hhk::ClassicSpec::matches(m->km) || hhk::CorticalSpec::matches(m->km))) return HH_E_UNSUPPORTED;
  hipStream_t s = (hipStream_t)stream;
  const size_t bytes = (size_t)m->km.n_gates * (size_t)n_nodes * sizeof(float4);
  if (m->d_tab && m->tab_n != n_nodes) {
    HIP_OK(hipStreamSynchronize(s));
    HIP_OK(hipFree(m->d_tab));
    m->d_tab = nullptr;
  }
  if (!m->d_tab && hipMalloc((void**)&m->d_tab, bytes) != hipSuccess) return HH_E_OOM;
  m->tab_n = n_nodes;
  m->tab_vlo = v_lo;
  // the lookup scale in binary32, and the nodes placed exactly where the
  // lookup puts them (v_lo + i / inv_h), so the step reads each node at the
  // voltage it was tabulated for
  m->tab_inv_h = (float)((double)(n_nodes - 1) / ((double)v_hi - (double)v_lo));
  HIP_OK(launch_build_table(m, s));
  return HH_OK;
}

int32_t hh_init_state(hh_model* m, float* state, const float* v0, float v0s, void* stream) {
  if (!m || !state) return HH_E_INVALID;
  HIP_OK(launch_init_state(m, state, v0, v0s, (hipStream_t)stream));
  return HH_OK;
}

int32_t hh_step_n(hh_model* m, float* state, int64_t t0, int32_t n_steps, const hh_input* in,
                  const hh_outputs* out, void* stream) {
  if (!m || !state) return HH_E_INVALID;
  if (n_steps < 0 || t0 < 0) return HH_E_SHAPE;
  hh_input none = {HH_IN_NONE, nullptr, 0.f, 0.f, 0, nullptr, 0.f, nullptr};
  hh_outputs nout = {nullptr, nullptr, nullptr, 1, nullptr};
  if (!in) in = &none;
  if (!out) out = &nout;
  if (in->mode < HH_IN_NONE || in->mode > HH_IN_SINE) return HH_E_INVALID;
  if (in->mode == HH_IN_SINE && (!in->i_const || !in->freq)) return HH_E_INVALID;
  if (in->mode == HH_IN_SINE && (m->row_ptr || m->d_cable)) return HH_E_UNSUPPORTED;
  if (in->mode == HH_IN_BACKGROUND && !(in->lam >= 0.0f && in->lam <= 80.0f)) return HH_E_INVALID;
  if (in->mode == HH_IN_CONST && !in->i_const) return HH_E_INVALID;
  if (in->mode == HH_IN_DENSE && !in->i_dense) return HH_E_INVALID;
  if (out->ckpt && out->ckpt_every < 1) return HH_E_SHAPE;
  if (m->d_tab && (m->row_ptr || !m->use_fixed)) return HH_E_UNSUPPORTED;
  if (m->d_cable && (m->row_ptr || out->ckpt || out->level)) return HH_E_UNSUPPORTED;
  if (m->row_ptr) return hh_net_step_n_internal(m, state, t0, n_steps, in, out, stream);
  if (n_steps == 0) return HH_OK;
  hipStream_t s = (hipStream_t)stream;
  StepArgs a;
  memset(&a, 0, sizeof(a));
  a.state = state;
  a.n = m->n;
  a.N = m->N;
  a.coef = m->coef;
  a.cm = m->cm;
  a.in_mode = in->mode;
  a.i_const = in->i_const;
  a.mu = in->mu;
  a.sigma = in->sigma;
  a.seed = in->seed;
  if (in->mode == HH_IN_BACKGROUND) {
    a.bg_lam = in->lam;
    a.bg_p0 = (float)exp(-(double)in->lam);
    a.bg_kmax = (int32_t)floor((double)in->lam + 12.0 * sqrt((double)in->lam)) + 12;
  }
  if (in->mode == HH_IN_SINE) {
    a.freq = in->freq;
    a.sine_K = (float)((double)m->km.dt * 4294967296.0 / 1000.0);
  }
  a.words = (m->n + 31) / 32;
  a.ckpt = out->ckpt;
  a.ckpt_every = out->ckpt ? out->ckpt_every : 1;
  a.level = out->level;
  a.bad = m->d_flags;
  if (m->d_tab) {
    a.tab = m->d_tab;
    a.tab_n = m->tab_n;
    a.tab_vlo = m->tab_vlo;
    a.tab_inv_h = m->tab_inv_h;
  }
  for (int32_t kb = 0; kb < n_steps; kb += m->k_fuse) {
    const int32_t ns = (n_steps - kb < m->k_fuse) ? n_steps - kb : m->k_fuse;
    a.t0 = t0 + kb;
    a.nsteps = ns;
    a.k_base = kb;
    a.i_dense = in->i_dense ? in->i_dense + (int64_t)kb * m->n : nullptr;
    a.spikes = out->spikes ? out->spikes + (int64_t)kb * a.words : nullptr;
    a.v_rec = out->v_rec ? out->v_rec + (int64_t)kb * m->n : nullptr;
    if (m->d_cable) {
      a.cable = m->d_cable;
      a.cable_K = m->cable_K;
      a.cable_D = m->cable_D;
      HIP_OK(launch_cable(m, a, s));
    } else {
      HIP_OK(launch_step(m, a, s));
    }
  }
  return HH_OK;
}

int32_t hh_check(hh_model* m, int64_t* first_bad, void* stream) {
  if (!m) return HH_E_INVALID;
  int32_t f[4];
  HIP_OK(hipStreamSynchronize((hipStream_t)stream));
  HIP_OK(hipMemcpy(f, m->d_flags, sizeof(f), hipMemcpyDeviceToHost));
  const int32_t reset[4] = {INT32_MAX, 0, 0, 0};
  HIP_OK(hipMemcpy(m->d_flags, reset, sizeof(reset), hipMemcpyHostToDevice));
  if (first_bad) *first_bad = (f[0] == INT32_MAX) ? -1 : f[0];
  if (f[1]) return HH_E_TIMEOUT;
  if (f[0] != INT32_MAX) return HH_E_NONFINITE;
  return HH_OK;
}

}  // extern "C"
