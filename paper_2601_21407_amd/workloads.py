"""Seeded synthetic workloads and model descriptions for the HH hot path.

This module holds model *descriptions* (channel tables as plain data) and
seeded input generators.  It contains none of the method's arithmetic: both
the HIP library and the FP64 oracle receive the dictionaries and arrays made
here and evaluate them with their own code.

Model dictionary format::

    {"gates":    [{"kind": "ab" | "inftau",
                   "rates": [(form, A, B, K, c), (form, A, B, K, c)]}, ...],
     "channels": [{"gbar": mS/cm^2, "E": mV, "gates": [(gate_index, exponent), ...]}, ...],
     "C": uF/cm^2, "dt": ms, "v_th": mV, "v_method": "fe" | "ee",
     "syn": None | {"tau_e": ms, "tau_i": ms, "E_e": mV, "E_i": mV}}

Rate forms (u = (V - B) / K): "exp" A e^u; "sigmoid" A / (1 + e^u);
"linoid" A (V - B) / (1 - e^{-u}); "bell" (c e^u + e^{-u}) / A.  A gate of
kind "ab" carries (alpha, beta) of Eq. (1); kind "inftau" carries (p_inf, 1/tau).
"""
from __future__ import annotations

import copy

import numpy as np


# ---------------------------------------------------------------------------
# channel tables
# ---------------------------------------------------------------------------
def _f32(x: float) -> float:
    """x as the nearest binary32 value (values beyond its range become
    infinite, as in the descriptor)."""
    with np.errstate(over="ignore"):
        return float(np.float32(x))


def binary32_model(model: dict) -> dict:
    """The model with every numeric parameter rounded to binary32.  The
    library's descriptor carries binary32 values, so a model is defined by
    those values: the oracle then integrates exactly the parameters the
    library integrates (0.1 and 0.3, for instance, differ from their binary32
    neighbours by up to 3e-8, coherently at every step)."""
    m = copy.deepcopy(model)
    for g in m["gates"]:
        g["rates"] = [(r[0],) + tuple(_f32(x) for x in r[1:]) for r in g["rates"]]
    for c in m["channels"]:
        c["gbar"], c["E"] = _f32(c["gbar"]), _f32(c["E"])
    for key in ("C", "dt", "v_th"):
        m[key] = _f32(m[key])
    if m.get("syn"):
        m["syn"] = {k: _f32(v) for k, v in m["syn"].items()}
    return m


def classic_hh(dt: float = 0.01, v_method: str = "fe", C: float = 1.0, syn=None) -> dict:
    """Hodgkin & Huxley (1952) squid axon in the modern -65 mV resting
    convention: Na (m^3 h, 120 mS/cm^2, +50 mV), K (n^4, 36, -77), leak
    (0.3, -54.4)."""
    return binary32_model({
        "gates": [
            {"kind": "ab", "rates": [("linoid", 0.1, -40.0, 10.0, 0.0), ("exp", 4.0, -65.0, -18.0, 0.0)]},
            {"kind": "ab", "rates": [("exp", 0.07, -65.0, -20.0, 0.0), ("sigmoid", 1.0, -35.0, -10.0, 0.0)]},
            {"kind": "ab", "rates": [("linoid", 0.01, -55.0, 10.0, 0.0), ("exp", 0.125, -65.0, -80.0, 0.0)]},
        ],
        "channels": [
            {"gbar": 120.0, "E": 50.0, "gates": [(0, 3), (1, 1)]},
            {"gbar": 36.0, "E": -77.0, "gates": [(2, 4)]},
            {"gbar": 0.3, "E": -54.4, "gates": []},
        ],
        "C": C, "dt": dt, "v_th": 0.0, "v_method": v_method, "syn": syn,
    })


V_T = -56.2  # spike-threshold offset of the cortical channel set


def custom_channels(dt: float = 0.025, v_method: str = "fe") -> dict:
    """Cortical channel set in the style of Pospischil et al. (2008): fast Na
    (m^3 h), delayed-rectifier K (n^4), slow M-type K (p, steady state and
    bell-shaped time constant), L-type Ca (q^2) and leak.  Conductances are
    this project's own choice, tuned so that 5 uA/cm^2 with noise fires
    tonically at about 20 Hz."""
    return binary32_model({
        "gates": [
            {"kind": "ab", "rates": [("linoid", 0.32, V_T + 13.0, 4.0, 0.0),
                                     ("linoid", -0.28, V_T + 40.0, -5.0, 0.0)]},
            {"kind": "ab", "rates": [("exp", 0.128, V_T + 17.0, -18.0, 0.0),
                                     ("sigmoid", 4.0, V_T + 40.0, -5.0, 0.0)]},
            {"kind": "ab", "rates": [("linoid", 0.032, V_T + 15.0, 5.0, 0.0),
                                     ("exp", 0.5, V_T + 10.0, -40.0, 0.0)]},
            {"kind": "inftau", "rates": [("sigmoid", 1.0, -35.0, -10.0, 0.0),
                                         ("bell", 1000.0, -35.0, 20.0, 3.3)]},
            {"kind": "ab", "rates": [("linoid", 0.055, -27.0, 3.8, 0.0),
                                     ("exp", 0.94, -75.0, -17.0, 0.0)]},
        ],
        "channels": [
            {"gbar": 50.0, "E": 50.0, "gates": [(0, 3), (1, 1)]},
            {"gbar": 6.0, "E": -90.0, "gates": [(2, 4)]},
            {"gbar": 0.3, "E": -90.0, "gates": [(3, 1)]},
            {"gbar": 0.1, "E": 120.0, "gates": [(4, 2)]},
            {"gbar": 0.15, "E": -70.0, "gates": []},
        ],
        "C": 1.0, "dt": dt, "v_th": 0.0, "v_method": v_method, "syn": None,
    })


def soma_dendrites(model: dict, n_dend: int = 3, per_dend: int = 5, g_axial: float = 1.5,
                   soma_area: float = 3.0, density: float = 0.3) -> dict:
    """Morphology description: a soma (compartment 0) with n_dend unbranched
    dendrites of per_dend compartments each, as in the paper's soma + three
    dendrites example (Results, sub-cellular scale).  Dendrites carry every
    channel of `model` at `density` times the soma's conductance (so their
    resting potential equals the soma's) and unit area; the soma has
    soma_area.  Every edge has conductance g_axial (mS/cm^2 per unit area).
    Returns {"K", "parent", "g_axial", "area", "gbar"} with K = 1 +
    n_dend * per_dend."""
    parent = [-1]
    for _ in range(n_dend):
        first = len(parent)
        parent.append(0)
        parent += list(range(first, first + per_dend - 1))
    K = len(parent)
    g0 = np.array([c["gbar"] for c in model["channels"]], dtype=np.float64)
    gbar = np.vstack([g0] + [density * g0] * (K - 1)).astype(np.float32).astype(np.float64)
    return {"K": K, "parent": parent, "g_axial": [0.0] + [_f32(g_axial)] * (K - 1),
            "area": [_f32(soma_area)] + [1.0] * (K - 1), "gbar": gbar}


def with_synapses(model: dict, tau_e=5.0, tau_i=10.0, E_e=0.0, E_i=-80.0) -> dict:
    m = copy.deepcopy(model)
    m["syn"] = {"tau_e": tau_e, "tau_i": tau_i, "E_e": E_e, "E_i": E_i}
    return binary32_model(m)


def coef_table(model: dict) -> np.ndarray:
    """Nominal rate coefficients as a [n_gates*8] float64 vector, index
    g*8 + r*4 + j for (A, B, K, c)."""
    G = len(model["gates"])
    out = np.zeros(G * 8)
    for g, gate in enumerate(model["gates"]):
        for r, rt in enumerate(gate["rates"]):
            out[g * 8 + r * 4: g * 8 + r * 4 + 4] = rt[1:5]
    return out


def jitter_coef(model: dict, n: int, seed: int, frac: float = 0.1, first: int = 0) -> np.ndarray:
    """Per-neuron rate coefficients, each nominal A, B, K, c multiplied by an
    independent factor uniform in [1 - frac, 1 + frac).  Returns float32
    [n_gates*8, n] for neurons first .. first+n-1 of the population (the
    factors of neuron i depend only on (seed, i))."""
    nom = coef_table(model)
    G = len(model["gates"])
    out = np.empty((G * 8, n), np.float32)
    block = 65536
    # generate in fixed blocks of neuron ids so a subset reproduces the same values
    b0, b1 = first // block, (first + n - 1) // block
    for b in range(b0, b1 + 1):
        rng = np.random.default_rng([seed, b])
        u = rng.random((G * 8, block))
        lo, hi = b * block, (b + 1) * block
        s0, s1 = max(lo, first), min(hi, first + n)
        fac = 1.0 + frac * (2.0 * u[:, s0 - lo: s1 - lo] - 1.0)
        out[:, s0 - first: s1 - first] = (nom[:, None] * fac).astype(np.float32)
    return out


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------
def validation_currents(n: int = 1024, seed: int = 1) -> np.ndarray:
    """Constant injected current per neuron, uniform in [0, 20) uA/cm^2."""
    return (20.0 * np.random.default_rng(seed).random(n)).astype(np.float32)


def net_csr(n: int = 38000, fan_out: int = 2630, frac_exc: float = 0.8, seed: int = 3,
            mu: float = -1.0, sigma: float = 0.5, inh_scale: float = 1.0):
    """Random recurrent connectivity: every source has exactly `fan_out`
    distinct non-self targets drawn uniformly, sorted; weights
    LogNormal(mu, sigma), stored negative (and multiplied by inh_scale) for
    inhibitory sources (ids >= frac_exc * n).  Returns (row_ptr int64 [n+1],
    col int32 [nnz], w float32 [nnz])."""
    rng = np.random.default_rng(seed)
    fan_out = min(fan_out, n - 1)
    nnz = n * fan_out
    col = np.empty(nnz, np.int32)
    chunk = max(1, min(n, (1 << 26) // max(n, 1)))
    for j0 in range(0, n, chunk):
        j1 = min(n, j0 + chunk)
        # distinct targets per row: top-k of uniform keys over the n-1 candidates
        keys = rng.random((j1 - j0, n - 1), dtype=np.float32)
        idx = np.argpartition(keys, fan_out - 1, axis=1)[:, :fan_out]
        idx.sort(axis=1)
        src = np.arange(j0, j1)[:, None]
        idx = idx + (idx >= src)  # skip the self connection
        col[j0 * fan_out: j1 * fan_out] = idx.reshape(-1).astype(np.int32)
    w = rng.lognormal(mu, sigma, nnz).astype(np.float32)
    n_exc = int(round(frac_exc * n))
    w[n_exc * fan_out:] *= -inh_scale
    row_ptr = np.arange(0, nnz + 1, fan_out, dtype=np.int64)
    return row_ptr, col, w


def net_external(n: int = 38000, frac: float = 0.01, rate_hz: float = 20.0, dt_ms: float = 0.1,
                 seed: int = 3):
    """Driven subset (mask) and the 32-bit event threshold floor(p * 2^32)
    for a Poisson drive of `rate_hz` sampled once per step."""
    rng = np.random.default_rng([seed, 7])
    k = int(round(frac * n))
    mask = np.zeros(n, np.uint8)
    mask[rng.choice(n, k, replace=False)] = 1
    p = rate_hz * dt_ms * 1e-3
    return mask, int(np.floor(p * 4294967296.0))


# Recurrent-network workload: 38,000 classic HH neurons (exponential Euler in
# V at dt = 0.1 ms), 80 % excitatory, 2,630 random targets per source,
# lognormal weights; conductance increment per spike = NET_W_SCALE * |w|
# (inhibitory weights NET_INH_SCALE times larger); 1 % of neurons receive
# 20 Hz Poisson events of NET_W_EXT.  The scale was calibrated once with the
# oracle for a mean rate near 10 Hz.
NET_W_SCALE = 0.03
NET_INH_SCALE = 4.0
NET_W_EXT = 0.5


def timescale_coef(model: dict, taus) -> np.ndarray:
    """Per-neuron rate coefficients [G*8][len(taus)] (the layout of
    coef_table) for neurons whose gate kinetics run tau times slower (the
    HH filter bank's time constant, Results, HH encryption): both rates of
    an (alpha, beta) gate and the 1/tau rate of a (p_inf, 1/tau) gate are
    divided by tau.  The amplitude is the coefficient A of the exp,
    sigmoid and linoid forms and 1/A of the bell form.  float32 values, the
    device's precision, handed to both sides."""
    base = coef_table(model).astype(np.float64)
    out = np.repeat(base[:, None], len(taus), axis=1)
    for g, gate in enumerate(model["gates"]):
        for r, rate in enumerate(gate["rates"]):
            if gate["kind"] != "ab" and r == 0:
                continue  # p_inf keeps its value
            row = g * 8 + r * 4
            for j, tau in enumerate(taus):
                out[row, j] = base[row] * tau if rate[0] == "bell" else base[row] / tau
    return out.astype(np.float32)


def pathway_delays(csr, n_pop: int = 8, max_delay: int = 15, seed: int = 21):
    """Per-synapse delays (steps, uint8 [nnz]) from a pathway table: the n
    neurons form n_pop equal contiguous populations, and every synapse from
    population a to population b carries the delay D[a][b], drawn once from
    U{1..max_delay}.  A synthetic stand-in for per-pathway delays (the
    published cortical tables are not available).  Returns (delays, D, pop)."""
    row_ptr, col = np.asarray(csr[0]), np.asarray(csr[1])
    n = len(row_ptr) - 1
    pop = (np.arange(n) * n_pop) // max(n, 1)
    D = np.random.default_rng([seed, 5]).integers(1, max_delay + 1, (n_pop, n_pop))
    src = np.repeat(np.arange(n), np.diff(row_ptr))
    return D[pop[src], pop[col]].astype(np.uint8), D, pop


def net_model() -> dict:
    return with_synapses(classic_hh(dt=0.1, v_method="ee"))


def net_v0(n: int, seed: int) -> np.ndarray:
    """Initial potentials uniform in [-70, -60) mV."""
    return (-70.0 + 10.0 * np.random.default_rng([seed, 11]).random(n)).astype(np.float32)


def layer_inputs(B: int = 256, T: int = 250, n_in: int = 700, n_cls: int = 20, seed: int = 4,
                 p: float = 0.02):
    """Synthetic spike sequences shaped like a 700-channel spoken-digit
    recording: class c fires channel ch at step t with probability
    p (1 + 0.9 sin(2 pi (f_c ch / n_in + g_c t / T) + phi_c)).  Returns
    (S uint8 [T, B, n_in], labels int64 [B])."""
    rng = np.random.default_rng(seed)
    f = rng.uniform(0.5, 3.0, n_cls)
    g = rng.uniform(0.5, 3.0, n_cls)
    phi = rng.uniform(0.0, 2 * np.pi, n_cls)
    labels = rng.integers(0, n_cls, B)
    ch = np.arange(n_in)[None, :]
    S = np.empty((T, B, n_in), np.uint8)
    for t in range(T):
        prob = p * (1.0 + 0.9 * np.sin(2 * np.pi * (f[labels, None] * ch / n_in
                                                   + g[labels, None] * t / T) + phi[labels, None]))
        S[t] = (rng.random((B, n_in)) < prob).astype(np.uint8)
    return S, labels.astype(np.int64)


def pack_bits(A) -> np.ndarray:
    """Binary matrix [M, K] (any dtype, values 0/1) to int32 words [M, ceil(K/32)]:
    bit k%32 of word k/32 is A[m, k]."""
    A = np.asarray(A) != 0
    M, K = A.shape
    wpr = (K + 31) // 32
    pad = np.zeros((M, wpr * 32), np.uint8)
    pad[:, :K] = A
    by = np.packbits(pad.reshape(M, wpr * 4, 8), axis=2, bitorder="little").reshape(M, wpr * 4)
    return np.ascontiguousarray(by).view(np.uint32).view(np.int32).reshape(M, wpr)


def pack_bits_cols(A) -> np.ndarray:
    """Binary matrix [M, K] to int32 words [ceil(M/32), K] packed along M:
    bit m%32 of word (m/32, k) is A[m, k] (the weight gradient's layout)."""
    A = np.asarray(A)
    if A.shape[0] == 0:
        return np.zeros((0, A.shape[1]), np.int32)
    return np.ascontiguousarray(pack_bits(A.T).T)


def layer_params(n_in: int = 700, H: int = 1024, n_cls: int = 20, seed: int = 4,
                 w_mean: float = 0.5, w_std: float = 0.8):
    """Initial parameters of the differentiable layer: W_in [n_in, H] (to be
    rounded to bf16 by the caller), per-unit C_m, readout W_out [H, n_cls], b."""
    rng = np.random.default_rng([seed, 1])
    W_in = (w_mean + w_std * rng.standard_normal((n_in, H))).astype(np.float32)
    W_out = (rng.standard_normal((H, n_cls)) / np.sqrt(H)).astype(np.float32)
    b = np.zeros(n_cls, np.float32)
    cm = np.ones(H, np.float32)
    return W_in, cm, W_out, b


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round float32 values to the nearest bfloat16 (ties to even), returned
    as float32."""
    a = np.ascontiguousarray(x, np.float32).view(np.uint32).astype(np.uint64)
    a = (a + 0x7FFF + ((a >> 16) & 1)) & 0xFFFF0000
    return a.astype(np.uint32).view(np.float32)
